// Register-row resident SB kernel (gfx950) and the spin ordering it uses.
//
// Paper section "Simulated Bifurcation": all K symplectic-Euler steps of
// bSB (Eq. 5-8) or dSB (Eq. 9-12) for one agent run inside one workgroup.
// Positions live in LDS (two buffers, kRegMaxN floats apart), momenta and
// each spin's couplings (column, J) live in VGPRs, so a step is: gather
// x_j for every held coupling, FMAs in CSR order, the update, one LDS
// store, one barrier.  Nothing touches HBM between the first and the last
// step.
//
// Spins are handed to threads in order of decreasing row length (thread t
// takes sorted positions t*SPT .. t*SPT+SPT-1), so the number of gathers a
// wave issues -- the longest row among its spins -- is small for almost
// every wave.  A spin's arithmetic does not depend on which thread runs
// it, so results are bit-identical to the streaming kernel.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

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

// Gather-and-sum over the first C held couplings of every slot: all LDS
// loads first, then the FMAs in CSR order onto acc (which enters holding
// h_i).  LDS holds what the coupling reads (x for bSB, sgn x for dSB).
// Entries past a row's length hold J = 0 and column 0: an exact zero
// contribution, since the running sum is never -0.
template <int SPT, int RC, int C>
__device__ __forceinline__ void reg_dots(const float *__restrict__ xc, const int (&cols)[SPT][RC],
                                         const float (&js)[SPT][RC], float (&acc)[SPT]) {
    float v[SPT][C];
#pragma unroll
    for (int s = 0; s < SPT; ++s)
#pragma unroll
        for (int e = 0; e < C; ++e) v[s][e] = xc[cols[s][e]];
#pragma unroll
    for (int s = 0; s < SPT; ++s) {
        float a = acc[s];
#pragma unroll
        for (int e = 0; e < C; ++e) a = __builtin_fmaf(js[s][e], v[s][e], a);
        acc[s] = a;
    }
}

template <int MODE, int MAXTPB, int SPT, int RC>
__global__ __launch_bounds__(MAXTPB) void sb_resident_reg(ResidentArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    float *xs = reinterpret_cast<float *>(smem);  // [2][kRegMaxN]
    double *red = reinterpret_cast<double *>(xs + 2 * kRegMaxN);
    const int n = A.n;
    const int t = threadIdx.x;
    const int m = blockIdx.x;
    const int M = A.M;

    float xr[SPT], yr[SPT], hr[SPT];
    int spin[SPT];
    int cols[SPT][RC];
    float js[SPT][RC];
    int tail0[SPT], tail1[SPT];
    int need = 0, tail = 0;
#pragma unroll
    for (int s = 0; s < SPT; ++s) {
        const int j = t * SPT + s;
        const int i = j < n ? A.perm[j] : -1;
        spin[s] = i;
        xr[s] = yr[s] = hr[s] = 0.0f;
        tail0[s] = tail1[s] = 0;
#pragma unroll
        for (int e = 0; e < RC; ++e) {
            cols[s][e] = 0;
            js[s][e] = 0.0f;
        }
        if (i >= 0) {
            const size_t o = static_cast<size_t>(i) * M + m;
            xr[s] = A.x[o];
            yr[s] = A.y[o];
            hr[s] = A.h[i];
            const int p0 = A.row_ptr[i], p1 = A.row_ptr[i + 1];
#pragma unroll
            for (int e = 0; e < RC; ++e) {
                if (p0 + e < p1) {
                    cols[s][e] = A.col[p0 + e];
                    js[s][e] = A.J[p0 + e];
                }
            }
            tail0[s] = p0 + RC;
            tail1[s] = p1;
            need = max(need, p1 - p0);
            tail |= (p1 - p0 > RC) ? 1 : 0;
            xs[i] = shared_value<MODE>(xr[s]);
        }
    }
    const int cap = wave_max_int(need);
    const int any_tail = wave_max_int(tail);
    __syncthreads();

    const float c0 = static_cast<float>(A.scal[0]);
    const float dt = A.dt, dta0 = A.dta0;
    int ck = 0;
    auto step = [&](auto bufc, int k) {
        constexpr int B = decltype(bufc)::value;
        const float *xc = xs + B * kRegMaxN;
        float *xn = xs + (B ^ 1) * kRegMaxN;
        const float g = A.sched[k];
        float acc[SPT];
#pragma unroll
        for (int s = 0; s < SPT; ++s) acc[s] = hr[s];
        if constexpr (RC <= 2) {
            reg_dots<SPT, RC, RC>(xc, cols, js, acc);
        } else if constexpr (RC <= 4) {
            if (cap <= 2)
                reg_dots<SPT, RC, 2>(xc, cols, js, acc);
            else
                reg_dots<SPT, RC, RC>(xc, cols, js, acc);
        } else {
            if (cap <= 2)
                reg_dots<SPT, RC, 2>(xc, cols, js, acc);
            else if (cap <= 4)
                reg_dots<SPT, RC, 4>(xc, cols, js, acc);
            else
                reg_dots<SPT, RC, RC>(xc, cols, js, acc);
        }
        if (any_tail) {
#pragma unroll
            for (int s = 0; s < SPT; ++s)
                for (int p = tail0[s]; p < tail1[s]; ++p)
                    acc[s] = __builtin_fmaf(A.J[p], xc[A.col[p]], acc[s]);
        }
#pragma unroll
        for (int s = 0; s < SPT; ++s) {
            if (spin[s] >= 0) {
                sb_update(xr[s], yr[s], acc[s], c0, g, dt, dta0);
                xn[spin[s]] = shared_value<MODE>(xr[s]);
            }
        }
        __syncthreads();
        if (A.ckpt_every > 0 && (k + 1) % A.ckpt_every == 0) {
            // FP64 O(T) of this agent's current state (Eq. 13)
            double e = 0.0;
#pragma unroll
            for (int s = 0; s < SPT; ++s) {
                const int i = spin[s];
                if (i >= 0 && xr[s] >= 0.0f) {
                    double er = A.a[i];
                    for (int p = A.row_ptr[i]; p < A.row_ptr[i + 1]; ++p) {
                        const int c = A.col[p];
                        if (c > i && xn[c] >= 0.0f) er += A.b[p];
                    }
                    e += er;
                }
            }
            const double tot = block_sum(e, red);
            if (t == 0) A.etrace[static_cast<size_t>(ck) * M + m] = tot;
            ++ck;
        }
    };
    int k = 0;
    for (; k + 1 < A.K; k += 2) {
        step(std::integral_constant<int, 0>{}, k);
        step(std::integral_constant<int, 1>{}, k + 1);
    }
    if (k < A.K) step(std::integral_constant<int, 0>{}, k);
#pragma unroll
    for (int s = 0; s < SPT; ++s) {
        const int i = spin[s];
        if (i >= 0) {
            const size_t o = static_cast<size_t>(i) * M + m;
            A.x[o] = xr[s];
            A.y[o] = yr[s];
        }
    }
}

hipError_t launch_row_order(int n, const int *row_ptr, int *perm, hipStream_t st) {
    row_order<<<1, 1024, 0, st>>>(n, row_ptr, perm);
    return hipGetLastError();
}

template <int MODE, int MAXTPB, int SPT>
static hipError_t launch_reg_rc(const ResidentArgs &A, const ResidentShape &S, hipStream_t st) {
    const dim3 grid(A.M), block(S.tpb);
    switch (S.rc) {
        case 2: return launch_with_lds(sb_resident_reg<MODE, MAXTPB, SPT, 2>, grid, block, S.lds_bytes, st, A);
        case 4: return launch_with_lds(sb_resident_reg<MODE, MAXTPB, SPT, 4>, grid, block, S.lds_bytes, st, A);
        case 8:
            if constexpr (SPT <= 4)
                return launch_with_lds(sb_resident_reg<MODE, MAXTPB, SPT, 8>, grid, block, S.lds_bytes, st, A);
            else
                return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

template <int MODE, int MAXTPB>
static hipError_t launch_reg_spt(const ResidentArgs &A, const ResidentShape &S, hipStream_t st) {
    switch (S.spt) {
        case 1: return launch_reg_rc<MODE, MAXTPB, 1>(A, S, st);
        case 2: return launch_reg_rc<MODE, MAXTPB, 2>(A, S, st);
        case 4: return launch_reg_rc<MODE, MAXTPB, 4>(A, S, st);
        case 8: return launch_reg_rc<MODE, MAXTPB, 8>(A, S, st);
        default: return hipErrorInvalidValue;
    }
}

template <int MODE>
static hipError_t launch_reg_m(const ResidentArgs &A, const ResidentShape &S, hipStream_t st) {
    if (S.tpb <= 0 || S.tpb % 64 != 0) return hipErrorInvalidValue;
    if (S.tpb <= 256) return launch_reg_spt<MODE, 256>(A, S, st);
    if (S.tpb <= 512) return launch_reg_spt<MODE, 512>(A, S, st);
    if (S.tpb <= 1024) return launch_reg_spt<MODE, 1024>(A, S, st);
    return hipErrorInvalidValue;
}

hipError_t launch_resident_reg(int mode, const ResidentArgs &A, const ResidentShape &S,
                               hipStream_t st) {
    return mode == kDSB ? launch_reg_m<kDSB>(A, S, st) : launch_reg_m<kBSB>(A, S, st);
}

}  // namespace sbt
