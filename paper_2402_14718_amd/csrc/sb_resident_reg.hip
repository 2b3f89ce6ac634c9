// Register-row resident SB kernel (gfx950): the spin ordering it uses and
// the dispatch to the step kernel of each mode (sb_resident_reg_step.hpp,
// built once per mode in sb_resident_reg_{bsb,dsb,asb}.hip).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sb_device.hpp"
#include "sb_kernels.hpp"

namespace sbt {

constexpr int kOrderClasses = 10;  // row lengths 0..8 and "9 or more"

// perm[0..n) = spins by decreasing min(row length, 9), ascending spin id
// within a length.  One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void row_order(int n, const int *__restrict__ row_ptr,
                                                  int *__restrict__ perm) {
    __shared__ int wave_tot[16];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    int base = 0;
    for (int cls = kOrderClasses - 1; cls >= 0; --cls) {
        for (int c0 = 0; c0 < n; c0 += 1024) {
            const int i = c0 + t;
            bool f = false;
            if (i < n) {
                const int len = row_ptr[i + 1] - row_ptr[i];
                f = min(len, kOrderClasses - 1) == cls;
            }
            const uint64_t bal = __ballot(f);
            const int below = __popcll(bal & ((uint64_t(1) << lane) - 1));
            if (lane == 0) wave_tot[wave] = __popcll(bal);
            __syncthreads();
            int woff = 0, tot = 0;
            for (int w = 0; w < 16; ++w) {
                woff += (w < wave) ? wave_tot[w] : 0;
                tot += wave_tot[w];
            }
            if (f) perm[base + woff + below] = i;
            base += tot;
            __syncthreads();
        }
    }
}

hipError_t launch_row_order(int n, const int *row_ptr, int *perm, hipStream_t st) {
    row_order<<<1, 1024, 0, st>>>(n, row_ptr, perm);
    return hipGetLastError();
}

hipError_t launch_resident_reg(int mode, const ResidentArgs &A, const ResidentShape &S,
                               hipStream_t st) {
    if (mode == kASB) return launch_resident_reg_asb(A, S, st);
    return mode == kDSB ? launch_resident_reg_dsb(A, S, st) : launch_resident_reg_bsb(A, S, st);
}

}  // namespace sbt
