// Register-row resident SB kernel (gfx950).
//
// Paper section "Simulated Bifurcation": all K symplectic-Euler steps of
// bSB (Eq. 5-8) or dSB (Eq. 9-12) for one agent run inside one workgroup.
// Positions live in LDS (two buffers, kRegStride floats apart), momenta and
// each spin's couplings (column, J) live in VGPRs, so a step is: gather
// x_j for every held coupling, FMAs in CSR order, the update, one LDS
// store, one barrier.  Nothing touches HBM between the first and the last
// step.
//
// Spins are handed out slot-major in order of decreasing row length (slot s
// of thread t takes sorted position s*T + t, T threads), so the few long
// rows sit in slot 0 of the first waves.  Each wave picks, once, a step
// loop with a fixed gather count for slot 0 and one for its other slots
// (the longest row it holds there), so a step has no branches.  Entries
// past a row's length hold J = 0 and column 0: adding them changes at most
// the sign of a zero sum, which never grows into a nonzero difference.  A
// spin's arithmetic does not depend on which thread runs it, so results are
// bit-identical to the streaming kernel.
//
// Register capacity: slot 0 holds up to RC couplings of its row, the other
// slots RR (RC, or 2 when RC everywhere does not fit the VGPR budget: slot
// 0 holds the longest rows).  Couplings past a slot's capacity are copied
// once into an LDS area at kernel start (placed by a block scan) and summed
// from there after the held ones, in CSR order; if they do not fit, from
// global memory.
//
// This header holds the step kernel and its shape dispatch;
// sb_resident_reg_{bsb,dsb,asb}.hip build one mode each (in parallel),
// sb_resident_reg.hip the spin order and the mode dispatch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "sb_device.hpp"
#include "sb_kernels.hpp"

namespace sbt {

// Calls f(integral_constant<int, C>) with C the smallest of 2, 4, RC that
// covers cap (cap is wave-uniform).
template <int RC, class F>
__device__ __forceinline__ void by_cap(int cap, F &&f) {
    if constexpr (RC <= 2) {
        f(std::integral_constant<int, RC>{});
    } else if constexpr (RC <= 4) {
        if (cap <= 2)
            f(std::integral_constant<int, 2>{});
        else
            f(std::integral_constant<int, RC>{});
    } else {
        if (cap <= 2)
            f(std::integral_constant<int, 2>{});
        else if (cap <= 4)
            f(std::integral_constant<int, 4>{});
        else
            f(std::integral_constant<int, RC>{});
    }
}

// RC couplings of slot 0's row are held in registers, RR of every other
// slot's (RR <= RC: slots past 0 hold the shorter rows).
template <int MODE, int MAXTPB, int SPT, int RC, int RR>
__global__ __launch_bounds__(MAXTPB) void sb_resident_reg(ResidentArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    float *xs = reinterpret_cast<float *>(smem);  // [2][kRegStride]
    double *red = reinterpret_cast<double *>(xs + 2 * kRegStride);  // [MAXTPB / 64]
    // couplings past a row's register capacity: [kRegTailCap] columns, values
    int *tcol = reinterpret_cast<int *>(red + MAXTPB / 64);
    float *tJ = reinterpret_cast<float *>(tcol + kRegTailCap);
    const int n = A.n;
    const int t = threadIdx.x;
    const int m = blockIdx.x;
    const int M = A.M;

    float xr[SPT], yr[SPT], hr[SPT];
    // LDS word each slot's position is stored to: the spin index, or a pad
    // word past every spin for a lane without one
    int wr[SPT];
    int cols[SPT][RC];
    float js[SPT][RC];
    int need0 = 0, need_rest = 0, rest = 0, tail = 0;
    int tlen[SPT];  // couplings of the slot's row past its capacity
#pragma unroll
    for (int s = 0; s < SPT; ++s) {
        const int j = s * static_cast<int>(blockDim.x) + t;
        const int i = j < n ? A.perm[j] : -1;
        // a lane without a spin in this slot updates a zero oscillator and
        // stores it to its own pad word, so the step has no branches
        wr[s] = i >= 0 ? i : kRegMaxN + (t & 63);
        xr[s] = yr[s] = hr[s] = 0.0f;
        tlen[s] = 0;
        const int cap = s == 0 ? RC : RR;
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
                if (e < cap && p0 + e < p1) {
                    cols[s][e] = A.col[p0 + e];
                    js[s][e] = A.J[p0 + e];
                }
            }
            if (s == 0) {
                need0 = p1 - p0;
            } else {
                need_rest = max(need_rest, p1 - p0);
                rest = 1;
            }
            tail |= (p1 - p0 > cap) ? 1 : 0;
            tlen[s] = max(0, p1 - p0 - cap);
            xs[i] = shared_value<MODE>(xr[s]);
        }
    }
    const int cap0 = wave_max_int(need0);
    const int cap_rest = wave_max_int(need_rest);
    const int any_rest = wave_max_int(rest);
    const int any_tail = wave_max_int(tail);
    // Tails are staged in LDS once (offsets by a block scan), each slot
    // keeping (offset << 12 | length) in one register; a kernel whose tails
    // do not fit reads them from global memory instead.
    int mine = 0;
#pragma unroll
    for (int s = 0; s < SPT; ++s) mine += tlen[s];
    int total = 0;
    const int before = block_exclusive_scan(mine, reinterpret_cast<int *>(red), total);
    const bool lds_tails = total <= kRegTailCap;
    int tpk[SPT];
    {
        int off = before;
#pragma unroll
        for (int s = 0; s < SPT; ++s) {
            tpk[s] = lds_tails ? (off << 12) | tlen[s] : 0;  // off, tlen < 2^11 here
            if (lds_tails && tlen[s] > 0) {
                const int i = wr[s];
                const int p = A.row_ptr[i] + (s == 0 ? RC : RR);
                for (int q = 0; q < tlen[s]; ++q) {
                    tcol[off + q] = A.col[p + q];
                    tJ[off + q] = A.J[p + q];
                }
            }
            off += tlen[s];
        }
    }
    __syncthreads();

    const float c0 = static_cast<float>(A.scal[0]);
    const float dt = A.dt, dta0 = A.dta0;

    // The whole step loop, specialised per wave: C0 gathers for slot 0, CR
    // for every other slot (0: this wave holds no spin past slot 0).  The
    // choice is made once, so a step runs straight through: gathers, FMAs
    // in CSR order, update, LDS store, barrier (rows longer than their
    // slot's capacity, rare, continue from global memory out of line).
    // Every variant meets the same barriers.
    auto run = [&](auto c0c, auto crc) __attribute__((always_inline)) {
        constexpr int C0 = decltype(c0c)::value;
        constexpr int CR = decltype(crc)::value;
        constexpr int NS = CR > 0 ? SPT : 1;  // slots this wave updates
        auto step = [&](auto bufc, int k) __attribute__((always_inline)) {
            constexpr int B = decltype(bufc)::value;
            const float *xc = xs + B * kRegStride;
            float *xn = xs + (B ^ 1) * kRegStride;
            const float g = A.sched[k];
            float acc[SPT];
            float v[SPT][RC];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                acc[s] = hr[s];
                const int C = s == 0 ? C0 : CR;
#pragma unroll
                for (int e = 0; e < C; ++e) v[s][e] = xc[cols[s][e]];
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int C = s == 0 ? C0 : CR;
#pragma unroll
                for (int e = 0; e < C; ++e) acc[s] = __builtin_fmaf(js[s][e], v[s][e], acc[s]);
            }
            if (__builtin_expect(any_tail, 0)) {
                if (lds_tails) {
#pragma unroll
                    for (int s = 0; s < NS; ++s)
                        for (int q = tpk[s] >> 12, q1 = q + (tpk[s] & 4095); q < q1; ++q)
                            acc[s] = __builtin_fmaf(tJ[q], xc[tcol[q]], acc[s]);
                } else {
#pragma unroll
                    for (int s = 0; s < NS; ++s)
                        for (int p = wr[s] < n ? A.row_ptr[wr[s]] + (s == 0 ? RC : RR) : 0,
                                 p1 = wr[s] < n ? A.row_ptr[wr[s] + 1] : 0;
                             p < p1; ++p)
                            acc[s] = __builtin_fmaf(A.J[p], xc[A.col[p]], acc[s]);
                }
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                sb_step<MODE>(xr[s], yr[s], acc[s], c0, g, dt, dta0);
                xn[wr[s]] = shared_value<MODE>(xr[s]);
            }
            __syncthreads();
        };
        // steps in runs between checkpoints; the buffer read at step k is k & 1
        int k = 0, ck = 0;
        while (k < A.K) {
            const int kend =
                A.ckpt_every > 0 ? min(A.K, k - k % A.ckpt_every + A.ckpt_every) : A.K;
            if (k & 1) step(std::integral_constant<int, 1>{}, k++);
            for (; k + 1 < kend; k += 2) {
                step(std::integral_constant<int, 0>{}, k);
                step(std::integral_constant<int, 1>{}, k + 1);
            }
            if (k < kend) step(std::integral_constant<int, 0>{}, k++);
            if (A.ckpt_every > 0 && k % A.ckpt_every == 0) {
                // FP64 O(T) of this agent's current state (Eq. 13)
                const float *xv = xs + (k & 1) * kRegStride;
                double e = 0.0;
#pragma unroll
                for (int s = 0; s < SPT; ++s) {
                    const int i = wr[s] < n ? wr[s] : -1;
                    if (i >= 0 && xr[s] >= 0.0f) {
                        double er = A.a[i];
                        for (int p = A.row_ptr[i]; p < A.row_ptr[i + 1]; ++p) {
                            const int c = A.col[p];
                            if (c > i && xv[c] >= 0.0f) er += A.b[p];
                        }
                        e += er;
                    }
                }
                const double tot = block_sum(e, red);
                if (t == 0) A.etrace[static_cast<size_t>(ck) * M + m] = tot;
                ++ck;
            }
        }
    };
    // rows past slot 0 are short: 2 gathers, else RR
    by_cap<RC>(cap0, [&](auto c0c) __attribute__((always_inline)) {
        if constexpr (SPT == 1) {
            run(c0c, std::integral_constant<int, 0>{});
        } else {
            if (!any_rest)
                run(c0c, std::integral_constant<int, 0>{});
            else if (RR <= 2 || cap_rest <= 2)
                run(c0c, std::integral_constant<int, 2>{});
            else
                run(c0c, std::integral_constant<int, RR>{});
        }
    });
#pragma unroll
    for (int s = 0; s < SPT; ++s) {
        const int i = wr[s] < n ? wr[s] : -1;
        if (i >= 0) {
            const size_t o = static_cast<size_t>(i) * M + m;
            A.x[o] = xr[s];
            A.y[o] = yr[s];
        }
    }
}

template <int MODE, int MAXTPB, int SPT, int RC, int RR>
hipError_t launch_reg_shape(const ResidentArgs &A, const ResidentShape &S, hipStream_t st) {
    if constexpr (reg_variant_fits(MAXTPB, SPT, RC, RR))
        return launch_with_lds(sb_resident_reg<MODE, MAXTPB, SPT, RC, RR>, dim3(A.M), dim3(S.tpb),
                               S.lds_bytes, st, A);
    else
        return hipErrorInvalidValue;
}

// only the shapes the host can pick are built
template <int MODE, int MAXTPB, int SPT>
hipError_t launch_reg_rc(const ResidentArgs &A, const ResidentShape &S, hipStream_t st) {
    const bool split = S.rr != S.rc;
    if (split && S.rr != 2) return hipErrorInvalidValue;
    switch (S.rc) {
        case 2: return launch_reg_shape<MODE, MAXTPB, SPT, 2, 2>(A, S, st);
        case 4:
            return split ? launch_reg_shape<MODE, MAXTPB, SPT, 4, 2>(A, S, st)
                         : launch_reg_shape<MODE, MAXTPB, SPT, 4, 4>(A, S, st);
        case 8:
            return split ? launch_reg_shape<MODE, MAXTPB, SPT, 8, 2>(A, S, st)
                         : launch_reg_shape<MODE, MAXTPB, SPT, 8, 8>(A, S, st);
        default: return hipErrorInvalidValue;
    }
}

template <int MODE, int MAXTPB>
hipError_t launch_reg_spt(const ResidentArgs &A, const ResidentShape &S, hipStream_t st) {
    switch (S.spt) {
        case 1: return launch_reg_rc<MODE, MAXTPB, 1>(A, S, st);
        case 2: return launch_reg_rc<MODE, MAXTPB, 2>(A, S, st);
        case 3: return launch_reg_rc<MODE, MAXTPB, 3>(A, S, st);
        case 4: return launch_reg_rc<MODE, MAXTPB, 4>(A, S, st);
        case 8: return launch_reg_rc<MODE, MAXTPB, 8>(A, S, st);
        default: return hipErrorInvalidValue;
    }
}

template <int MODE>
hipError_t launch_reg_m(const ResidentArgs &A, const ResidentShape &S, hipStream_t st) {
    if (S.tpb <= 0 || S.tpb % 64 != 0) return hipErrorInvalidValue;
    if (S.tpb <= 256) return launch_reg_spt<MODE, 256>(A, S, st);
    if (S.tpb <= 512) return launch_reg_spt<MODE, 512>(A, S, st);
    if (S.tpb <= 1024) return launch_reg_spt<MODE, 1024>(A, S, st);
    return hipErrorInvalidValue;
}


}  // namespace sbt
