// Streaming bSB / aSB step over row quads (gfx950).
//
// Same step as sb_stream_v4 (paper section "Simulated Bifurcation", Eq. 5-8
// and Eq. 1-4) and bit-identical to it; what differs is how the neighbours'
// positions are gathered.  Every coupling reads x_j for all agents, and that
// gathered volume (nnz x agents x 4 bytes) is what binds the streaming step:
// it all passes through each CU's vector-memory path.  In the azimuth spin
// order consecutive rows share many neighbours, so a wave here takes four
// consecutive rows (a quad) at once: once per solve the quad's distinct
// columns are listed in ascending order with, for each, the coupling of
// each of the four rows (0 where a row has none), and each step the wave
// gathers x_j once per listed column and applies it to all four rows.  Each
// row's sum is still seeded with h_i and taken in ascending column order
// (the absent couplings add exact zeros), as in the CSR step.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sb_device.hpp"
#include "sb_kernels.hpp"
#include "sb_stream_kernels.hpp"
#include "sb_stream_chunk.hpp"

namespace sbt {

namespace {

constexpr int kR = kQuadRows;
constexpr int kChunk = kStreamChunk;
constexpr int kScanThreads = 1024;
typedef float f32x4 __attribute__((ext_vector_type(4)));

// A stored coupling of the padded rows decoded to FP32 exactly as the CSR
// streaming step decodes it.
template <int JP>
__device__ __forceinline__ float stored_coupling(const StreamArgs &A, int p, int row) {
    if constexpr (JP == kJFp8)
        return A.rowscale[row] * e4m3_to_f32<0>(A.J8[p]);
    else if constexpr (JP == kJFp8Blk)
        return A.blkscale[p / kChunk] * e4m3_to_f32<0>(A.J8[p]);
    else if constexpr (JP == kJBf16x2)
        return bf16x2_value(A.J2[p]);
    else
        return A.J[p];
}

// Walks the union of the quad's rows (padded CSR; a row's own column marks
// its padding) in ascending column order, calling f(column, p[kR]) with
// p[r] the row's entry for that column or -1.
template <class F>
__device__ __forceinline__ void quad_union(int n, const int *prow, const int *pcol, int quad, F &&f) {
    int pos[kR], end[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int i = quad * kR + r;
        pos[r] = i < n ? prow[i] : 0;
        end[r] = i < n ? prow[i + 1] : 0;
        while (pos[r] < end[r] && pcol[end[r] - 1] == i) --end[r];  // drop the padding
    }
    while (true) {
        int c = INT32_MAX;
#pragma unroll
        for (int r = 0; r < kR; ++r)
            if (pos[r] < end[r]) c = min(c, pcol[pos[r]]);
        if (c == INT32_MAX) break;
        int at[kR];
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            at[r] = -1;
            if (pos[r] < end[r] && pcol[pos[r]] == c) at[r] = pos[r]++;
        }
        f(c, at);
    }
}

__global__ __launch_bounds__(256) void quad_count(int n, int nq, const int *__restrict__ prow,
                                                  const int *__restrict__ pcol, int *__restrict__ cnt) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= nq) return;
    int d = 0;
    quad_union(n, prow, pcol, q, [&](int, const int *) { ++d; });
    cnt[q] = (d + kChunk - 1) / kChunk * kChunk;
}

// cnt[0..nq) -> qoff[0..nq] (exclusive prefix sums, qoff[nq] = total); one
// workgroup, each thread a contiguous range.
__global__ __launch_bounds__(kScanThreads) void quad_scan(int nq, const int *__restrict__ cnt,
                                                          int *__restrict__ qoff) {
    __shared__ int tot[kScanThreads];
    const int t = threadIdx.x;
    const int per = (nq + kScanThreads - 1) / kScanThreads;
    const int q0 = min(nq, t * per), q1 = min(nq, q0 + per);
    int sum = 0;
    for (int q = q0; q < q1; ++q) sum += cnt[q];
    tot[t] = sum;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {
        const int v = t >= d ? tot[t - d] : 0;
        __syncthreads();
        tot[t] += v;
        __syncthreads();
    }
    int at = tot[t] - sum;
    for (int q = q0; q < q1; ++q) {
        qoff[q] = at;
        at += cnt[q];
    }
    if (t == kScanThreads - 1) qoff[nq] = tot[t];
}

template <int JP>
__global__ __launch_bounds__(256) void quad_fill(int nq, StreamArgs A, const int *__restrict__ qoff,
                                                 int *__restrict__ qcol, float *__restrict__ qJ) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= nq) return;
    int u = qoff[q];
    const int u1 = qoff[q + 1];
    int last = 0;
    quad_union(A.n, A.row_ptr, A.col, q, [&](int c, const int *at) {
        qcol[u] = c;
#pragma unroll
        for (int r = 0; r < kR; ++r)
            qJ[static_cast<size_t>(u) * kR + r] = at[r] >= 0 ? stored_coupling<JP>(A, at[r], q * kR + r) : 0.0f;
        last = c;
        ++u;
    });
    for (; u < u1; ++u) {  // padding to whole chunks: a listed column, no coupling
        qcol[u] = last;
#pragma unroll
        for (int r = 0; r < kR; ++r) qJ[static_cast<size_t>(u) * kR + r] = 0.0f;
    }
}

// Workgroup id -> (quad block, agent block), XCD-contiguous: each XCD
// sweeps one contiguous range of quads (neighbouring quads share lines).
__device__ __forceinline__ bool quad_block(int nqb, int nab, int &qb, int &ab) {
    const int total = nqb * nab;
    const int per_xcd = (total + 7) / 8;
    const int v = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (v >= total) return false;
    ab = v / nqb;
    qb = v % nqb;
    return true;
}

}  // namespace

// One step: a wave = one quad x 256 agents (four per lane).
template <int MODE, bool NT>
__global__ __launch_bounds__(256) void sb_stream_quad(StreamArgs A, int k, const int *__restrict__ qoff,
                                                      const int *__restrict__ qcol,
                                                      const float *__restrict__ qJ,
                                                      const float *__restrict__ h,
                                                      const float *__restrict__ xin,
                                                      float *__restrict__ xout, float *__restrict__ y) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int M = A.M;
    const int nq = (A.n + kR - 1) / kR;
    const int nqb = (nq + 3) / 4;
    const int nab = (M + 255) / 256;
    int qb, ab;
    if (!quad_block(nqb, nab, qb, ab)) return;
    const int q = __builtin_amdgcn_readfirstlane(qb * 4 + wave);
    if (q >= nq) return;
    const int i0 = q * kR;
    const int m = ab * 256 + 4 * lane;
    const bool live = m < M;
    const int mcol = live ? m : 0;  // dead lanes read agents 0..3 (in bounds)
    const float c0 = static_cast<float>(A.scal[0]);
    const float g = A.sched[k];
    float4 acc[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const float hv = i0 + r < A.n ? h[i0 + r] : 0.0f;
        acc[r] = make_float4(hv, hv, hv, hv);
    }
    const int u1 = qoff[q + 1];
    for (int u = qoff[q]; u < u1; u += kChunk) {
        const int4 ca = *reinterpret_cast<const int4 *>(qcol + u);
        const int4 cb = *reinterpret_cast<const int4 *>(qcol + u + 4);
        const int c[kChunk] = {ca.x, ca.y, ca.z, ca.w, cb.x, cb.y, cb.z, cb.w};
        float w[kChunk][kR];
#pragma unroll
        for (int e = 0; e < kChunk; ++e)
#pragma unroll
            for (int r = 0; r < kR; ++r) w[e][r] = qJ[static_cast<size_t>(u + e) * kR + r];
        float4 v[kChunk];
#pragma unroll
        for (int e = 0; e < kChunk; ++e)
            v[e] = *reinterpret_cast<const float4 *>(xin + static_cast<size_t>(c[e]) * M + mcol);
#pragma unroll
        for (int e = 0; e < kChunk; ++e)
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                acc[r].x = __builtin_fmaf(w[e][r], v[e].x, acc[r].x);
                acc[r].y = __builtin_fmaf(w[e][r], v[e].y, acc[r].y);
                acc[r].z = __builtin_fmaf(w[e][r], v[e].z, acc[r].z);
                acc[r].w = __builtin_fmaf(w[e][r], v[e].w, acc[r].w);
            }
    }
    if (!live) return;
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        if (i0 + r >= A.n) break;
        const size_t o = static_cast<size_t>(i0 + r) * M + mcol;
        const f32x4 xv = ld_stream<NT>(reinterpret_cast<const f32x4 *>(xin + o));
        const f32x4 yv = ld_stream<NT>(reinterpret_cast<const f32x4 *>(y + o));
        float x[4] = {xv.x, xv.y, xv.z, xv.w}, yy[4] = {yv.x, yv.y, yv.z, yv.w};
        const float f[4] = {acc[r].x, acc[r].y, acc[r].z, acc[r].w};
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            if constexpr (MODE == kASB)
                sb_update_asb(x[a], yy[a], f[a], c0, g, A.dt, A.dta0);
            else
                sb_update(x[a], yy[a], f[a], c0, g, A.dt, A.dta0);
        }
        st_stream<NT>(f32x4{x[0], x[1], x[2], x[3]}, reinterpret_cast<f32x4 *>(xout + o));
        st_stream<NT>(f32x4{yy[0], yy[1], yy[2], yy[3]}, reinterpret_cast<f32x4 *>(y + o));
    }
}

size_t quad_cols_bound(int n, int64_t nnz) {
    const size_t nq = (static_cast<size_t>(n) + kR - 1) / kR;
    return static_cast<size_t>(nnz) + (kChunk - 1) * nq;
}

hipError_t launch_quad_plan(int jprec, const StreamArgs &A, const QuadArgs &Q, hipStream_t st) {
    const int nq = (A.n + kR - 1) / kR;
    const unsigned g = static_cast<unsigned>((nq + 255) / 256);
    quad_count<<<g, 256, 0, st>>>(A.n, nq, A.row_ptr, A.col, Q.qcnt);
    quad_scan<<<1, kScanThreads, 0, st>>>(nq, Q.qcnt, Q.qoff);
    switch (jprec) {
        case kJFp8: quad_fill<kJFp8><<<g, 256, 0, st>>>(nq, A, Q.qoff, Q.qcol, Q.qJ); break;
        case kJFp8Blk: quad_fill<kJFp8Blk><<<g, 256, 0, st>>>(nq, A, Q.qoff, Q.qcol, Q.qJ); break;
        case kJBf16x2: quad_fill<kJBf16x2><<<g, 256, 0, st>>>(nq, A, Q.qoff, Q.qcol, Q.qJ); break;
        case kJFp32: quad_fill<kJFp32><<<g, 256, 0, st>>>(nq, A, Q.qoff, Q.qcol, Q.qJ); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_stream_quad(int mode, const StreamArgs &A, const QuadArgs &Q, int k, const float *xin,
                              float *xout, hipStream_t st) {
    if (A.M % 4 != 0) return hipErrorInvalidValue;
    const int nq = (A.n + kR - 1) / kR;
    const int total = (nq + 3) / 4 * ((A.M + 255) / 256);
    const dim3 grid((total + 7) / 8 * 8);
    const bool nt = static_cast<size_t>(A.n) * A.M * sizeof(float) * 3 > (size_t(256) << 20);
    if (mode == kASB) {
        if (nt)
            sb_stream_quad<kASB, true><<<grid, 256, 0, st>>>(A, k, Q.qoff, Q.qcol, Q.qJ, A.h, xin, xout, A.y);
        else
            sb_stream_quad<kASB, false><<<grid, 256, 0, st>>>(A, k, Q.qoff, Q.qcol, Q.qJ, A.h, xin, xout, A.y);
    } else if (mode == kBSB) {
        if (nt)
            sb_stream_quad<kBSB, true><<<grid, 256, 0, st>>>(A, k, Q.qoff, Q.qcol, Q.qJ, A.h, xin, xout, A.y);
        else
            sb_stream_quad<kBSB, false><<<grid, 256, 0, st>>>(A, k, Q.qoff, Q.qcol, Q.qJ, A.h, xin, xout, A.y);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace sbt
