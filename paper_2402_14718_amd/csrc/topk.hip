// sbt_top_k_dev: the k lowest FP64 agent energies and their agents, in
// ascending order, on the GPU -- the readout of the best agents (paper
// section "Results": the lowest energy over the shots; the stress workload
// reports its best 32).  One workgroup; the j-th pick is the least
// (energy, agent) pair greater than the (j-1)-th, so nothing is marked or
// sorted in place and ties go to the lower agent, as in the argmin of the
// solves.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "common.hpp"
#include "sbtrack.h"

namespace {

constexpr int kT = 1024;
constexpr int kNone = 0x7fffffff;  // no pair held yet

// Total order on (energy, agent): NaN after every number, then the agent.
__device__ __forceinline__ bool less_pair(double e1, int a1, double e2, int a2) {
    const bool n1 = e1 != e1, n2 = e2 != e2;
    if (n1 != n2) return n2;
    if (!n1 && e1 != e2) return e1 < e2;
    return a1 < a2;
}

__global__ __launch_bounds__(kT) void top_k_select(const double *__restrict__ energy, int agents,
                                                   int k, double *__restrict__ top_energy,
                                                   int *__restrict__ top_agent) {
    __shared__ double se[kT / 64];
    __shared__ int sa[kT / 64];
    __shared__ double last_e;
    __shared__ int last_a;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    for (int j = 0; j < k; ++j) {
        const double pe = j > 0 ? last_e : 0.0;
        const int pa = j > 0 ? last_a : -1;
        double be = NAN;
        int ba = kNone;
        for (int m = t; m < agents; m += kT) {
            const double e = energy[m];
            if ((j == 0 || less_pair(pe, pa, e, m)) && (ba == kNone || less_pair(e, m, be, ba))) {
                be = e;
                ba = m;
            }
        }
        for (int off = 32; off >= 1; off >>= 1) {
            const double oe = __shfl_xor(be, off, 64);
            const int oa = __shfl_xor(ba, off, 64);
            if (oa != kNone && (ba == kNone || less_pair(oe, oa, be, ba))) {
                be = oe;
                ba = oa;
            }
        }
        if (lane == 0) {
            se[wave] = be;
            sa[wave] = ba;
        }
        __syncthreads();
        if (t == 0) {
            for (int w = 1; w < kT / 64; ++w)
                if (sa[w] != kNone && (ba == kNone || less_pair(se[w], sa[w], be, ba))) {
                    be = se[w];
                    ba = sa[w];
                }
            top_energy[j] = be;
            top_agent[j] = ba;
            last_e = be;
            last_a = ba;
        }
        __syncthreads();
    }
}

}  // namespace

extern "C" int sbt_top_k_dev(const double *energy, int32_t agents, int32_t k, double *top_energy,
                             int32_t *top_agent, void *stream) {
    const char *who = "sbt_top_k_dev";
    sbt::clear_error();
    if (!energy || !top_energy || !top_agent) return sbt::fail(SBT_EINVAL, "%s: NULL argument", who);
    if (agents < 1) return sbt::fail(SBT_EINVAL, "%s: agents must be >= 1", who);
    if (k < 1 || k > agents) return sbt::fail(SBT_EINVAL, "%s: k = %d outside 1..%d", who, k, agents);
    top_k_select<<<1, kT, 0, static_cast<hipStream_t>(stream)>>>(energy, agents, k, top_energy,
                                                                 top_agent);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return sbt::fail(SBT_EDEVICE, "%s: launch: %s", who, hipGetErrorString(e));
    return SBT_OK;
}
