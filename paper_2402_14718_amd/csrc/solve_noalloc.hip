// sbt_solve_dev_noalloc: sbt_solve_dev with its scratch memory in a
// fixed-size array the library owns on each device, for callers that must
// not allocate (code under HIP graph capture, serving loops, harnesses that
// forbid hipMalloc).  The kernels are those of sbt_solve_dev; only where
// the workspace lives differs.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "common.hpp"
#include "sbtrack.h"

namespace {

// The workspace of every no-allocation solve on a device: 64 MiB, held by
// each device the library runs on until the process ends.  Every call on a
// device uses the same array, so calls that overlap on one device race.
constexpr size_t kScratchBytes = size_t(64) << 20;
static_assert(kScratchBytes == SBT_NOALLOC_SCRATCH_BYTES, "header and library disagree");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_lock;
void *g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current.  (In host code the array's name is a
// host-side stand-in, not a device address.)
int scratch_on_current_device(void **out, const char *who) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return sbt::fail(SBT_EDEVICE, "%s: hipGetDevice: %s", who, hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return sbt::fail(SBT_EUNSUPPORTED, "%s: device %d beyond the %d supported", who, dev, kMaxDevices);
    std::lock_guard<std::mutex> g(g_lock);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return sbt::fail(SBT_EDEVICE, "%s: hipGetSymbolAddress(scratch): %s", who,
                             hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return SBT_OK;
}

}  // namespace

extern "C" int sbt_solve_dev_noalloc(const sbt_dev_qubo *q, int32_t max_row_nnz, sbt_mode mode,
                                     const sbt_solve_params *p, const sbt_dev_result *out,
                                     void *stream) {
    const char *who = "sbt_solve_dev_noalloc";
    sbt::clear_error();
    if (!q || !p || !out) return sbt::fail(SBT_EINVAL, "%s: NULL argument", who);
    // the size check needs no device, so an oversized request fails before
    // any HIP call
    const size_t need = sbt_workspace_bytes(q->n, q->nnz, mode, p);
    if (need == 0) return SBT_EINVAL;  // message set by sbt_workspace_bytes
    if (need > kScratchBytes)
        return sbt::fail(SBT_EINVAL,
                         "%s: this solve needs %zu bytes of scratch, above the %zu-byte limit "
                         "(use sbt_solve_dev with a caller workspace)",
                         who, need, kScratchBytes);
    void *ws = nullptr;
    const int rc = scratch_on_current_device(&ws, who);
    if (rc) return rc;
    return sbt_solve_dev(q, max_row_nnz, mode, p, ws, kScratchBytes, out, stream);
}
