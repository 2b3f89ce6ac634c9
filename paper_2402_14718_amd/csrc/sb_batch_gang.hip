// Events of a batch that are too large for one workgroup's slots, run as
// gangs of row bands (gfx950).
//
// Same method as the batch step kernel (section "Simulated Bifurcation":
// bSB Eq. 5-8, dSB Eq. 9-12, aSB Eq. 1-4) and the same arithmetic per
// (spin, agent): the field seeds the sum, couplings follow in CSR order as
// 16-bit values, the fused update of sb_device.hpp.  A gang is one (event,
// agent): its spins are cut into `bands` runs of at most `rows` consecutive
// spins, one work item each, and all bands of a gang run at once on
// different workgroups of a persistent grid (items are queued gang after
// gang, and the grid is at least as large as any gang, so the bands of the
// gang being started are always taken by running workgroups).  Each step
// every band reads its neighbours' shared values (x, or sgn x for dSB) from
// the gang's position buffer of that step, writes its own into the other
// buffer, and meets the other bands at a barrier (an arrival counter).
//
// The XCDs' L2 caches are not coherent with each other inside a launch, so
// the buffers are read and written with agent-scope atomic loads and
// stores (coherent at the device level), and every thread fences at agent
// scope before its workgroup arrives.  Every wait is bounded by the device
// wall clock: a gang whose barrier does not fill within kWaitTicks sets
// gang_fault and stops waiting (its results are then meaningless; the host
// reports the flag), so every wave reaches the end of the kernel.
// In target mode a gang stops at the first checkpoint whose energy (the sum
// of its bands' parts) reaches the event's target.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>

#include "sb_device.hpp"
#include "sb_kernels.hpp"

namespace sbt {

namespace {

constexpr int kGT = 1024;                  // threads per gang workgroup
constexpr int kGS = kBatchSPT;             // spins per thread (rows <= kGT * kGS)
constexpr long long kWaitTicks = 1000000000LL;  // 10 s at the 100 MHz wall clock

template <int JP>
__device__ __forceinline__ float j16(uint16_t bits) {
    if constexpr (JP == kJFp16)
        return static_cast<float>(__ushort_as_half(bits));
    else
        return __uint_as_float(static_cast<uint32_t>(bits) << 16);
}

__device__ __forceinline__ float load_shared(const float *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_shared(float *p, float v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Arrive at the gang's barrier `phase` (1, 2, ...) and wait until all its
// bands have; every thread of the workgroup calls it.
__device__ void gang_barrier(int *arrive, int bands, int phase, int *fault) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(arrive, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const long long t0 = wall_clock64();
        while (__hip_atomic_load(arrive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
               bands * phase) {
            if (__hip_atomic_load(fault, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
            if (wall_clock64() - t0 > kWaitTicks) {
                __hip_atomic_store(fault, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

}  // namespace

template <int MODE, int JP>
__global__ __launch_bounds__(kGT) void sb_batch_gang(BatchArgs B) {
    __shared__ int item_s, stop_s;
    __shared__ double red[kGT / 64];
    const int t = threadIdx.x;
    for (;;) {
        if (t == 0) item_s = atomicAdd(B.gang_counter, 1);
        __syncthreads();
        const int item = item_s;
        __syncthreads();
        if (item >= B.gang_items) return;
        const GangDesc G = B.gangs[B.gitem_gang[item]];
        const int band = B.gitem_band[item];
        const BatchEvent E = B.ev[G.e];
        const int i0 = band * G.rows;
        const int i1 = min(E.n, i0 + G.rows);
        float *xb0 = B.xg + G.x_off, *xb1 = xb0 + E.n;
        int *arrive = B.arrive + (B.gitem_gang[item]);
        const int pstride = B.n_ckpt + 1;
        double *part = B.gpart + G.part_off + static_cast<size_t>(band) * pstride;
        long long *clk = B.gclock + G.part_off + static_cast<size_t>(band) * pstride;
        if (t == 0) clk[0] = wall_clock64();
        const float c0 = B.c0[G.e];

        float xr[kGS], yr[kGS], hr[kGS];
#pragma unroll
        for (int s = 0; s < kGS; ++s) {
            const int i = i0 + s * kGT + t;
            xr[s] = yr[s] = hr[s] = 0.0f;
            if (i < i1) {
                const Philox4 r = philox4x32_10(static_cast<uint32_t>(i), static_cast<uint32_t>(G.agent),
                                                static_cast<uint32_t>(E.event_id), 0u, B.seed_lo,
                                                B.seed_hi);
                xr[s] = philox_word_to_unit(r.v[0]);
                yr[s] = philox_word_to_unit(r.v[1]);
                hr[s] = B.h[E.row_off + i];
                store_shared(xb0 + i, shared_value<MODE>(xr[s]));
            }
        }
        int phase = 1;
        gang_barrier(arrive, G.bands, phase++, B.gang_fault);

        // FP64 energy of this band's rows (Eq. 13, pairs j > i) of the
        // positions in xv, summed over the workgroup in a fixed order
        auto band_energy = [&](const float *xv) -> double {
            double v = 0.0;
#pragma unroll
            for (int s = 0; s < kGS; ++s) {
                const int i = i0 + s * kGT + t;
                if (i < i1 && xr[s] >= 0.0f) {
                    double er = B.a[E.row_off + i];
                    const int p1 = B.row_ptr[E.rp_off + i + 1];
                    for (int p = B.row_ptr[E.rp_off + i]; p < p1; ++p) {
                        const int c = B.col[E.nz_off + p];
                        if (c > i && load_shared(xv + c) >= 0.0f) er += B.b[E.nz_off + p];
                    }
                    v += er;
                }
            }
            v = wave_sum(v);
            if ((t & 63) == 0) red[t >> 6] = v;
            __syncthreads();
            double tot = 0.0;
            if (t == 0)
                for (int w = 0; w < kGT / 64; ++w) tot += red[w];
            __syncthreads();
            return tot;
        };

        const float dt = B.dt, dta0 = B.dta0;
        int ck = 0, k_done = B.K;
        for (int k = 0; k < B.K; ++k) {
            const float *xin = (k & 1) ? xb1 : xb0;
            float *xout = (k & 1) ? xb0 : xb1;
            const float g = B.sched[k];
#pragma unroll
            for (int s = 0; s < kGS; ++s) {
                const int i = i0 + s * kGT + t;
                if (i < i1) {
                    float acc = hr[s];
                    const int p1 = B.row_ptr[E.rp_off + i + 1];
                    for (int p = B.row_ptr[E.rp_off + i]; p < p1; ++p)
                        acc = __builtin_fmaf(j16<JP>(B.J16[E.nz_off + p]),
                                             load_shared(xin + B.col[E.nz_off + p]), acc);
                    sb_step<MODE>(xr[s], yr[s], acc, c0, g, dt, dta0);
                    store_shared(xout + i, shared_value<MODE>(xr[s]));
                }
            }
            gang_barrier(arrive, G.bands, phase++, B.gang_fault);
            if (B.ckpt_every > 0 && (k + 1) % B.ckpt_every == 0 && ck < B.n_ckpt) {
                const double en = band_energy(xout);
                if (t == 0) {
                    __hip_atomic_store(part + ck, en, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    clk[ck + 1] = wall_clock64();
                }
                ++ck;
                if (B.target) {
                    // target mode: every band sums all bands' parts in band
                    // order, so all take the same decision
                    gang_barrier(arrive, G.bands, phase++, B.gang_fault);
                    if (t == 0) {
                        const double *p0 = B.gpart + G.part_off;
                        double tot = 0.0;
                        for (int b = 0; b < G.bands; ++b)
                            tot += __hip_atomic_load(p0 + static_cast<size_t>(b) * pstride + ck - 1,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        stop_s = tot <= B.target[G.e];
                    }
                    __syncthreads();
                    if (stop_s) {
                        k_done = k + 1;
                        break;
                    }
                }
            }
        }
        if (t == 0)
            for (int c = ck; c < B.n_ckpt; ++c) {  // checkpoints a target stop skipped
                part[c] = NAN;
                clk[c + 1] = 0;
            }
        const float *xfin = (k_done & 1) ? xb1 : xb0;
        const double en = band_energy(xfin);
        if (t == 0) part[B.n_ckpt] = en;
#pragma unroll
        for (int s = 0; s < kGS; ++s) {
            const int i = i0 + s * kGT + t;
            if (i < i1) {
                const size_t o = (static_cast<size_t>(E.row_off) + i) * B.M + G.agent;
                B.T[o] = xr[s] >= 0.0f ? 1 : 0;
                if (B.x_out) B.x_out[o] = xr[s];
            }
        }
    }
}

// Per gang: the energies (sum of its bands' partials in band order; NaN if
// a gang wait timed out), the checkpoint energies and stamps (the last
// band's stamp: when every part is known; the first band's start).
__global__ void batch_gang_reduce(BatchArgs B, int n_gangs) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_gangs) return;
    const GangDesc G = B.gangs[g];
    const int ps = B.n_ckpt + 1;
    // a gang whose barrier timed out has no meaningful energies
    const bool faulted = *B.gang_fault != 0;
    for (int c = 0; c <= B.n_ckpt; ++c) {
        double tot = faulted ? NAN : 0.0;
        long long last = 0;
        for (int b = 0; b < G.bands; ++b) {
            tot += B.gpart[G.part_off + b * ps + c];
            if (c < B.n_ckpt) last = max(last, B.gclock[G.part_off + b * ps + c + 1]);
        }
        if (c < B.n_ckpt) {
            B.etrace[(static_cast<size_t>(G.e) * B.n_ckpt + c) * B.M + G.agent] = tot;
            if (B.ckpt_clock)
                B.ckpt_clock[(static_cast<size_t>(G.e) * ps + c + 1) * B.M + G.agent] = last;
        } else {
            B.energy[static_cast<size_t>(G.e) * B.M + G.agent] = tot;
        }
    }
    if (B.ckpt_clock) {
        long long first = B.gclock[G.part_off];
        for (int b = 1; b < G.bands; ++b) first = min(first, B.gclock[G.part_off + b * ps]);
        B.ckpt_clock[(static_cast<size_t>(G.e) * ps) * B.M + G.agent] = first;
    }
}

__global__ void zero_ints(int *p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

hipError_t launch_batch_gang(int mode, int jprec, const BatchArgs &B, hipStream_t st) {
    const bool f16 = jprec == kJFp16;
    const dim3 grid(B.grid), block(kGT);
    if (mode == kDSB) {
        if (f16)
            sb_batch_gang<kDSB, kJFp16><<<grid, block, 0, st>>>(B);
        else
            sb_batch_gang<kDSB, kJBf16><<<grid, block, 0, st>>>(B);
    } else if (mode == kASB) {
        if (f16)
            sb_batch_gang<kASB, kJFp16><<<grid, block, 0, st>>>(B);
        else
            sb_batch_gang<kASB, kJBf16><<<grid, block, 0, st>>>(B);
    } else {
        if (f16)
            sb_batch_gang<kBSB, kJFp16><<<grid, block, 0, st>>>(B);
        else
            sb_batch_gang<kBSB, kJBf16><<<grid, block, 0, st>>>(B);
    }
    return hipGetLastError();
}

hipError_t launch_batch_gang_reduce(const BatchArgs &B, int n_gangs, hipStream_t st) {
    batch_gang_reduce<<<(n_gangs + 255) / 256, 256, 0, st>>>(B, n_gangs);
    return hipGetLastError();
}

hipError_t launch_zero_ints(int *p, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    zero_ints<<<(n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024, 256, 0, st>>>(p, n);
    return hipGetLastError();
}

}  // namespace sbt
