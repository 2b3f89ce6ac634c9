// Batched SB over many events (gfx950): per-event preparation, the work
// counters, best-agent selection, and the dispatch to the step kernel of
// each mode, coupling format and workgroup shape (sb_batch_step.hpp,
// instantiated once per triple by sb_batch_mode.hip).
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>

#include "sb_device.hpp"
#include "sb_kernels.hpp"

namespace sbt {

// Per-event preparation, one workgroup per event: FP32 field h, 16-bit
// couplings J = -b/4, c0 and the Ising offset C (FP64, fixed order), and
// the spin order by decreasing row length.
__global__ __launch_bounds__(256) void batch_prep(BatchArgs B, int jprec) {
    __shared__ double red[4];
    __shared__ int wave_tot[4];
    const int e = blockIdx.x;
    const BatchEvent E = B.ev[e];
    const int t = threadIdx.x;
    double sj = 0.0, sj2 = 0.0, sup = 0.0, sa = 0.0;
    for (int i = t; i < E.n; i += 256) {
        const int r0 = B.row_ptr[E.rp_off + i], r1 = B.row_ptr[E.rp_off + i + 1];
        double rs = 0.0;
        for (int p = r0; p < r1; ++p) {
            const double bv = B.b[E.nz_off + p];
            const double jv = -0.25 * bv;
            uint16_t bits;
            if (jprec == kJFp16) {
                bits = __half_as_ushort(static_cast<__half>(static_cast<_Float16>(jv)));
            } else {  // BF16: FP32 first, then round to nearest even on the upper half
                const uint32_t u = __float_as_uint(static_cast<float>(jv));
                bits = static_cast<uint16_t>((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
            }
            B.J16[E.nz_off + p] = bits;
            rs += bv;
            sj += jv;
            sj2 += jv * jv;
            if (B.col[E.nz_off + p] > i) sup += bv;
        }
        B.h[E.row_off + i] = static_cast<float>(-(0.5 * B.a[E.row_off + i] + 0.25 * rs));
        sa += B.a[E.row_off + i];
    }
    const double t0 = block_sum(sj, red);
    const double t1 = block_sum(sj2, red);
    const double t2 = block_sum(sup, red);
    const double t3 = block_sum(sa, red);
    if (t == 0) {
        const double n2 = static_cast<double>(E.n) * E.n;
        const double mean = t0 / n2;
        const double var = t1 / n2 - mean * mean;
        const double sd = var > 0.0 ? sqrt(var) : 0.0;
        double c0 = B.c0_fixed > 0.0 ? B.c0_fixed
                                     : (sd == 0.0 ? 0.5 / sqrt(static_cast<double>(E.n))
                                                  : 0.5 / (sqrt(static_cast<double>(E.n)) * sd));
        B.c0[e] = static_cast<float>(c0 * static_cast<double>(E.c0_scale));
        B.offset[e] = 0.5 * t3 + 0.25 * t2;
    }
    // spin order: decreasing min(row length, 63), ascending id within a length
    const int lane = t & 63, wave = t >> 6;
    int base = 0;
    for (int cls = 63; cls >= 0; --cls) {
        for (int c0i = 0; c0i < E.n; c0i += 256) {
            const int i = c0i + t;
            bool f = false;
            if (i < E.n) {
                const int len = B.row_ptr[E.rp_off + i + 1] - B.row_ptr[E.rp_off + i];
                f = min(len, 63) == cls;
            }
            const uint64_t bal = __ballot(f);
            const int below = __popcll(bal & ((uint64_t(1) << lane) - 1));
            if (lane == 0) wave_tot[wave] = __popcll(bal);
            __syncthreads();
            int woff = 0, tot = 0;
            for (int w = 0; w < 4; ++w) {
                woff += (w < wave) ? wave_tot[w] : 0;
                tot += wave_tot[w];
            }
            if (f) B.perm[E.row_off + base + woff + below] = i;
            base += tot;
            __syncthreads();
        }
    }
}

__global__ void batch_reset(int *counters, int n) {
    if (static_cast<int>(threadIdx.x) < n) counters[threadIdx.x] = 0;
}

// Per event: best agent (minimum energy, lowest index on ties), its T,
// and the best-so-far trace over checkpoints.
__global__ __launch_bounds__(256) void batch_select(BatchArgs B) {
    __shared__ double se[256];
    __shared__ int sm[256];
    const int e = blockIdx.x, t = threadIdx.x;
    const BatchEvent E = B.ev[e];
    double be = INFINITY;
    int bm = 0x7fffffff;
    for (int m = t; m < B.M; m += 256) {
        const double v = B.energy[static_cast<size_t>(e) * B.M + m];
        if (v < be || (v == be && m < bm)) {
            be = v;
            bm = m;
        }
    }
    se[t] = be;
    sm[t] = bm;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (t < w && (se[t + w] < se[t] || (se[t + w] == se[t] && sm[t + w] < sm[t]))) {
            se[t] = se[t + w];
            sm[t] = sm[t + w];
        }
        __syncthreads();
    }
    const int best = sm[0];
    if (t == 0) {
        B.best_energy[e] = se[0];
        B.best_agent[e] = best;
    }
    if (best >= 0 && best < B.M)
        for (int i = t; i < E.n; i += 256)
            B.best_T[E.row_off + i] = B.T[(static_cast<size_t>(E.row_off) + i) * B.M + best];
    if (B.trace && B.n_ckpt > 0) {
        double bsf = INFINITY;
        for (int c = 0; c < B.n_ckpt; ++c) {
            double v = INFINITY;
            for (int m = t; m < B.M; m += 256)
                v = fmin(v, B.etrace[(static_cast<size_t>(e) * B.n_ckpt + c) * B.M + m]);
            se[t] = v;
            __syncthreads();
            for (int w = 128; w >= 1; w >>= 1) {
                if (t < w) se[t] = fmin(se[t], se[t + w]);
                __syncthreads();
            }
            bsf = fmin(bsf, se[0]);
            if (t == 0) B.trace[static_cast<size_t>(e) * B.n_ckpt + c] = bsf;
            __syncthreads();
        }
    }
}

hipError_t launch_batch_prep(int jprec, const BatchArgs &B, hipStream_t st) {
    batch_prep<<<B.E, 256, 0, st>>>(B, jprec);
    return hipGetLastError();
}

hipError_t launch_batch_reset(int *counters, int n, hipStream_t st) {
    batch_reset<<<1, 64, 0, st>>>(counters, n);
    return hipGetLastError();
}

template <int TPB>
static hipError_t steps_of_shape(int mode, int jprec, const BatchArgs &B, hipStream_t st) {
    const bool f16 = jprec == kJFp16;
    if (mode == kDSB)
        return f16 ? launch_batch_steps_tu<kDSB, kJFp16, TPB>(B, st)
                   : launch_batch_steps_tu<kDSB, kJBf16, TPB>(B, st);
    if (mode == kASB)
        return f16 ? launch_batch_steps_tu<kASB, kJFp16, TPB>(B, st)
                   : launch_batch_steps_tu<kASB, kJBf16, TPB>(B, st);
    return f16 ? launch_batch_steps_tu<kBSB, kJFp16, TPB>(B, st)
               : launch_batch_steps_tu<kBSB, kJBf16, TPB>(B, st);
}

hipError_t launch_batch_steps(int mode, int jprec, int tpb, const BatchArgs &B, hipStream_t st) {
    if (tpb == kBatchTPBSmall) return steps_of_shape<kBatchTPBSmall>(mode, jprec, B, st);
    if (tpb == kBatchTPB) return steps_of_shape<kBatchTPB>(mode, jprec, B, st);
    return hipErrorInvalidValue;
}

hipError_t launch_batch_select(const BatchArgs &B, hipStream_t st) {
    batch_select<<<B.E, 256, 0, st>>>(B);
    return hipGetLastError();
}

}  // namespace sbt
