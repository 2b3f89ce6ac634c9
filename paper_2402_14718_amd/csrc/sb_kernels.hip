// Simulated-bifurcation kernels for gfx950 (CDNA4).
//
// Paper section "Simulated Bifurcation": bSB (Eq. 5-8) and dSB (Eq. 9-12)
// integrated with the symplectic Euler method, every spin and every agent
// updated in parallel.  Kernels here:
//
//   prep_ising_rows / prep_finalize   QUBO (FP64) -> J = -b/4 (FP32),
//                                     h = -(a/2 + rowsum(b)/4) (FP32),
//                                     C, c0 (FP64, fixed-order reductions)
//   init_state                        Philox4x32-10 start x0, y0
//   sb_resident<MODE, TPB, SPT, JLDS> all K steps in one launch: one
//                                     workgroup per agent, positions in LDS
//                                     (ping-pong), momenta in VGPRs, J in
//                                     LDS when it fits
//   (the streaming one-step kernel is in sb_stream.hip)
//   energy_rows / energy_reduce       FP64 O(T) of every agent (Eq. 13)
//   select_best                       argmin over agents (lowest index on
//                                     ties) and the best T
//   trace_reduce                      best-so-far O(T) per checkpoint
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <unordered_map>

#include "sb_device.hpp"
#include "sb_kernels.hpp"

namespace sbt {

bool lds_attribute_needed(const void *fn, size_t lds) {
    static std::mutex mu;
    static std::unordered_map<const void *, size_t> opened;
    std::lock_guard<std::mutex> lock(mu);
    size_t &have = opened[fn];
    if (lds <= have) return false;
    have = lds;
    return true;
}

// ------------------------------------------------------------ Ising prep

// One thread per row: J = -b/4 in FP32, h_i = -(a_i/2 + 1/4 sum_j b_ij),
// and per-block partial sums {sum J, sum J^2, sum_{j>i} b, sum a} in FP64.
__global__ __launch_bounds__(256) void prep_ising_rows(int n, const double *__restrict__ a,
                                                       const int *__restrict__ row_ptr,
                                                       const int *__restrict__ col,
                                                       const double *__restrict__ b,
                                                       float *__restrict__ J,
                                                       float *__restrict__ h,
                                                       double *__restrict__ part) {
    __shared__ double red[4];
    const int i = blockIdx.x * 256 + threadIdx.x;
    double sj = 0.0, sj2 = 0.0, sup = 0.0, sa = 0.0;
    if (i < n) {
        double rs = 0.0;
        for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            const double bv = b[p];
            const double jv = -0.25 * bv;
            J[p] = static_cast<float>(jv);
            rs += bv;
            sj += jv;
            sj2 += jv * jv;
            if (col[p] > i) sup += bv;
        }
        h[i] = static_cast<float>(-(0.5 * a[i] + 0.25 * rs));
        sa = a[i];
    }
    const double t0 = block_sum(sj, red);
    const double t1 = block_sum(sj2, red);
    const double t2 = block_sum(sup, red);
    const double t3 = block_sum(sa, red);
    if (threadIdx.x == 0) {
        part[4 * blockIdx.x + 0] = t0;
        part[4 * blockIdx.x + 1] = t1;
        part[4 * blockIdx.x + 2] = t2;
        part[4 * blockIdx.x + 3] = t3;
    }
}

// scal[0] = c0, scal[1] = C, scal[2] = sum J, scal[3] = sum J^2.
// c0 = 0.5 / (sqrt(N) sd(J)) with sd over all N^2 entries, unless the
// caller fixed c0 (> 0).
__global__ __launch_bounds__(256) void prep_finalize(int n, int nblk, double c0_fixed,
                                                     const double *__restrict__ part,
                                                     double *__restrict__ scal) {
    __shared__ double red[4];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    // each thread sums a strided subset in order, then a fixed tree
    for (int k = threadIdx.x; k < nblk; k += 256)
        for (int c = 0; c < 4; ++c) v[c] += part[4 * k + c];
    double t[4];
    for (int c = 0; c < 4; ++c) t[c] = block_sum(v[c], red);
    if (threadIdx.x == 0) {
        const double n2 = static_cast<double>(n) * static_cast<double>(n);
        const double mean = t[0] / n2;
        const double var = t[1] / n2 - mean * mean;
        const double sd = var > 0.0 ? sqrt(var) : 0.0;
        double c0;
        if (c0_fixed > 0.0)
            c0 = c0_fixed;
        else if (sd == 0.0)
            c0 = 0.5 / sqrt(static_cast<double>(n));
        else
            c0 = 0.5 / (sqrt(static_cast<double>(n)) * sd);
        scal[0] = c0;
        scal[1] = 0.5 * t[3] + 0.25 * t[2];
        scal[2] = t[0];
        scal[3] = t[1];
    }
}

// ------------------------------------------------------------ init state

__global__ __launch_bounds__(256) void init_state(int n, int M, uint32_t k0, uint32_t k1,
                                                  uint32_t event, float *__restrict__ x,
                                                  float *__restrict__ y) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (idx >= static_cast<int64_t>(n) * M) return;
    const uint32_t i = static_cast<uint32_t>(idx / M);
    const uint32_t m = static_cast<uint32_t>(idx % M);
    const Philox4 r = philox4x32_10(i, m, event, 0u, k0, k1);
    x[idx] = philox_word_to_unit(r.v[0]);
    y[idx] = philox_word_to_unit(r.v[1]);
}

// ------------------------------------------------------- schedule table

// sched[k] = a0 - a_k with a_k = a0 k / K (linear ramp from zero), FP64
// evaluated and rounded once to FP32; every step kernel reads this table.
__global__ __launch_bounds__(256) void schedule_table(int K, double a0, float *__restrict__ sched) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k < K) sched[k] = schedule_gap(a0, k, K);
}

// ------------------------------------------------------ resident kernel

// Workgroup = one agent, all n spins.  Thread t owns spins t, t+TPB, ...
// (SPT of them) and keeps their x, y, h and row bounds in registers; the
// positions every thread gathers from live in LDS, double-buffered so one
// barrier per step suffices.  LDS: [2][n] floats, then (JLDS) row_ptr,
// col, J, then the reduction scratch.
template <int MODE, int TPB, int SPT, bool JLDS>
__global__ __launch_bounds__(TPB) void sb_resident(ResidentArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = A.n;
    float *xs = reinterpret_cast<float *>(smem);
    int *s_rp = reinterpret_cast<int *>(xs + 2 * n);
    int *s_col = s_rp + (JLDS ? n + 1 : 0);
    float *s_J = reinterpret_cast<float *>(s_col + (JLDS ? A.nnz : 0));
    double *red = reinterpret_cast<double *>(
        (reinterpret_cast<uintptr_t>(s_J + (JLDS ? A.nnz : 0)) + 15) & ~uintptr_t(15));

    const int t = threadIdx.x;
    const int m = blockIdx.x;
    const int M = A.M;
    if constexpr (JLDS) {
        for (int k = t; k <= n; k += TPB) s_rp[k] = A.row_ptr[k];
        for (int k = t; k < A.nnz; k += TPB) {
            s_col[k] = A.col[k];
            s_J[k] = A.J[k];
        }
    }
    const int *cl = JLDS ? s_col : A.col;
    const float *jv = JLDS ? s_J : A.J;

    float xr[SPT], yr[SPT], hr[SPT];
    int p0[SPT], p1[SPT];
#pragma unroll
    for (int s = 0; s < SPT; ++s) {
        const int i = t + s * TPB;
        xr[s] = yr[s] = hr[s] = 0.0f;
        p0[s] = p1[s] = 0;
        if (i < n) {
            const size_t o = static_cast<size_t>(i) * M + m;
            xr[s] = A.x[o];
            yr[s] = A.y[o];
            hr[s] = A.h[i];
            p0[s] = A.row_ptr[i];
            p1[s] = A.row_ptr[i + 1];
            xs[i] = shared_value<MODE>(xr[s]);
        }
    }
    __syncthreads();

    const float c0 = static_cast<float>(A.scal[0]);
    const float dt = A.dt, dta0 = A.dta0;
    int cur = 0, ck = 0;
    float g_next = A.sched[0];  // loaded one step ahead
    for (int k = 0; k < A.K; ++k) {
        const float g = g_next;
        g_next = A.sched[min(k + 1, A.K - 1)];
        const float *xc = xs + cur * n;
        float *xn = xs + (cur ^ 1) * n;
#pragma unroll
        for (int s = 0; s < SPT; ++s) {
            const int i = t + s * TPB;
            if (i < n) {
                float acc = hr[s];
                for (int p = p0[s]; p < p1[s]; ++p) acc = __builtin_fmaf(jv[p], xc[cl[p]], acc);
                sb_step<MODE>(xr[s], yr[s], acc, c0, g, dt, dta0);
                xn[i] = shared_value<MODE>(xr[s]);
            }
        }
        __syncthreads();
        cur ^= 1;
        if (A.ckpt_every > 0 && (k + 1) % A.ckpt_every == 0) {
            // FP64 O(T) of this agent's current state (Eq. 13)
            const float *xv = xs + cur * n;
            double e = 0.0;
#pragma unroll
            for (int s = 0; s < SPT; ++s) {
                const int i = t + s * TPB;
                if (i < n && xr[s] >= 0.0f) {
                    double er = A.a[i];
                    for (int p = p0[s]; p < p1[s]; ++p) {
                        const int c = cl[p];
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
#pragma unroll
    for (int s = 0; s < SPT; ++s) {
        const int i = t + s * TPB;
        if (i < n) {
            const size_t o = static_cast<size_t>(i) * M + m;
            A.x[o] = xr[s];
            A.y[o] = yr[s];
        }
    }
}

// -------------------------------------------------------------- energy

// part[blockIdx.x * M + m] = sum over rows of this block of
// T_i (a_i + sum_{j > i} b_ij T_j) for agent m, T = (x >= 0).
__global__ __launch_bounds__(256) void energy_rows(int n, int M, int rows_per_block,
                                                   const double *__restrict__ a,
                                                   const int *__restrict__ row_ptr,
                                                   const int *__restrict__ col,
                                                   const double *__restrict__ b,
                                                   const float *__restrict__ x,
                                                   double *__restrict__ part) {
    __shared__ double red[4][64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int m = blockIdx.y * 64 + lane;
    const int r0 = blockIdx.x * rows_per_block;
    const int r1 = min(n, r0 + rows_per_block);
    double e = 0.0;
    if (m < M) {
        for (int r = r0 + wave; r < r1; r += 4) {
            const int i = __builtin_amdgcn_readfirstlane(r);
            if (x[static_cast<size_t>(i) * M + m] >= 0.0f) {
                double er = a[i];
                for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
                    const int c = col[p];
                    if (c > i && x[static_cast<size_t>(c) * M + m] >= 0.0f) er += b[p];
                }
                e += er;
            }
        }
    }
    red[wave][lane] = e;
    __syncthreads();
    if (wave == 0 && m < M)
        part[static_cast<size_t>(blockIdx.x) * M + m] =
            ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

__global__ __launch_bounds__(256) void energy_reduce(int nblk, int M, const double *__restrict__ part,
                                                     double *__restrict__ out) {
    const int m = blockIdx.x * 256 + threadIdx.x;
    if (m >= M) return;
    double e = 0.0;
    for (int k = 0; k < nblk; ++k) e += part[static_cast<size_t>(k) * M + m];
    out[m] = e;
}

// Best agent (minimum energy, lowest index on ties) and its T.
__global__ __launch_bounds__(1024) void select_best(int n, int M, const double *__restrict__ E,
                                                    const float *__restrict__ x,
                                                    double *__restrict__ best_e,
                                                    int *__restrict__ best_m,
                                                    int8_t *__restrict__ T) {
    __shared__ double se[1024];
    __shared__ int sm[1024];
    const int t = threadIdx.x;
    double be = INFINITY;
    int bm = 0x7fffffff;
    for (int m = t; m < M; m += 1024) {
        const double e = E[m];
        if (e < be || (e == be && m < bm)) {
            be = e;
            bm = m;
        }
    }
    se[t] = be;
    sm[t] = bm;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
        if (t < w) {
            const double e2 = se[t + w];
            const int m2 = sm[t + w];
            if (e2 < se[t] || (e2 == se[t] && m2 < sm[t])) {
                se[t] = e2;
                sm[t] = m2;
            }
        }
        __syncthreads();
    }
    const int mb = sm[0];
    if (t == 0) {
        *best_e = se[0];
        *best_m = mb;
    }
    if (mb < 0 || mb >= M) return;
    for (int i = t; i < n; i += 1024) T[i] = x[static_cast<size_t>(i) * M + mb] >= 0.0f ? 1 : 0;
}

// trace[c] = min(trace[c-1], min_m etrace[c, m]).
__global__ __launch_bounds__(256) void trace_reduce(int n_ckpt, int M, const double *__restrict__ et,
                                                    double *__restrict__ trace) {
    __shared__ double s[256];
    double bsf = INFINITY;
    for (int c = 0; c < n_ckpt; ++c) {
        double v = INFINITY;
        for (int m = threadIdx.x; m < M; m += 256) v = fmin(v, et[static_cast<size_t>(c) * M + m]);
        s[threadIdx.x] = v;
        __syncthreads();
        for (int w = 128; w >= 1; w >>= 1) {
            if (threadIdx.x < w) s[threadIdx.x] = fmin(s[threadIdx.x], s[threadIdx.x + w]);
            __syncthreads();
        }
        bsf = fmin(bsf, s[0]);
        if (threadIdx.x == 0) trace[c] = bsf;
        __syncthreads();
    }
}

// ------------------------------------------------------------ launchers

hipError_t launch_prep(int n, const double *a, const int *row_ptr, const int *col, const double *b,
                       float *J, float *h, double *part, double *scal, double c0_fixed,
                       hipStream_t st) {
    const int nblk = (n + 255) / 256;
    prep_ising_rows<<<nblk, 256, 0, st>>>(n, a, row_ptr, col, b, J, h, part);
    prep_finalize<<<1, 256, 0, st>>>(n, nblk, c0_fixed, part, scal);
    return hipGetLastError();
}

hipError_t launch_schedule(int K, double a0, float *sched, hipStream_t st) {
    schedule_table<<<(K + 255) / 256, 256, 0, st>>>(K, a0, sched);
    return hipGetLastError();
}

hipError_t launch_init(int n, int M, uint64_t seed, uint32_t event, float *x, float *y,
                       hipStream_t st) {
    const int64_t total = static_cast<int64_t>(n) * M;
    const int64_t blocks = (total + 255) / 256;
    init_state<<<static_cast<unsigned>(blocks), 256, 0, st>>>(
        n, M, static_cast<uint32_t>(seed & 0xffffffffu), static_cast<uint32_t>(seed >> 32), event,
        x, y);
    return hipGetLastError();
}

template <int MODE, int TPB, bool JLDS>
static hipError_t launch_lds_spt(const ResidentArgs &A, const ResidentShape &S, hipStream_t st) {
    switch (S.spt) {
        case 1: return launch_with_lds(sb_resident<MODE, TPB, 1, JLDS>, dim3(A.M), dim3(TPB), S.lds_bytes, st, A);
        case 2: return launch_with_lds(sb_resident<MODE, TPB, 2, JLDS>, dim3(A.M), dim3(TPB), S.lds_bytes, st, A);
        case 4: return launch_with_lds(sb_resident<MODE, TPB, 4, JLDS>, dim3(A.M), dim3(TPB), S.lds_bytes, st, A);
        case 8: return launch_with_lds(sb_resident<MODE, TPB, 8, JLDS>, dim3(A.M), dim3(TPB), S.lds_bytes, st, A);
        case 16: return launch_with_lds(sb_resident<MODE, TPB, 16, JLDS>, dim3(A.M), dim3(TPB), S.lds_bytes, st, A);
        default: return hipErrorInvalidValue;
    }
}

template <int MODE>
static hipError_t launch_resident_m(const ResidentArgs &A, const ResidentShape &S, hipStream_t st) {
    switch (S.tpb) {
        case 64: return S.jlds ? launch_lds_spt<MODE, 64, true>(A, S, st) : launch_lds_spt<MODE, 64, false>(A, S, st);
        case 256: return S.jlds ? launch_lds_spt<MODE, 256, true>(A, S, st) : launch_lds_spt<MODE, 256, false>(A, S, st);
        case 1024: return S.jlds ? launch_lds_spt<MODE, 1024, true>(A, S, st) : launch_lds_spt<MODE, 1024, false>(A, S, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_resident(int mode, const ResidentArgs &A, const ResidentShape &S, hipStream_t st) {
    if (S.rc > 0) return launch_resident_reg(mode, A, S, st);
    if (mode == kASB) return launch_resident_m<kASB>(A, S, st);
    return mode == kDSB ? launch_resident_m<kDSB>(A, S, st) : launch_resident_m<kBSB>(A, S, st);
}

hipError_t launch_energy(int n, int M, const double *a, const int *row_ptr, const int *col,
                         const double *b, const float *x, double *part, double *out,
                         hipStream_t st) {
    const int nblk = (n + kEnergyRows - 1) / kEnergyRows;
    dim3 grid(nblk, (M + 63) / 64);
    energy_rows<<<grid, 256, 0, st>>>(n, M, kEnergyRows, a, row_ptr, col, b, x, part);
    energy_reduce<<<(M + 255) / 256, 256, 0, st>>>(nblk, M, part, out);
    return hipGetLastError();
}

hipError_t launch_select_best(int n, int M, const double *E, const float *x, double *best_e,
                              int *best_m, int8_t *T, hipStream_t st) {
    select_best<<<1, 1024, 0, st>>>(n, M, E, x, best_e, best_m, T);
    return hipGetLastError();
}

hipError_t launch_trace_reduce(int n_ckpt, int M, const double *et, double *trace,
                               hipStream_t st) {
    trace_reduce<<<1, 256, 0, st>>>(n_ckpt, M, et, trace);
    return hipGetLastError();
}

}  // namespace sbt
