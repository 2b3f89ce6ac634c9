// Streaming bSB / aSB step with each row tile's neighbour positions staged
// in LDS (gfx950).
//
// Same step as sb_stream_v4 (paper section "Simulated Bifurcation", Eq. 5-8
// and Eq. 1-4): one launch per step, the coupling sum of each row seeded
// with h_i and taken over its padded CSR row in order, the fused update of
// sb_device.hpp -- so the results are bit-identical to it.  What differs is
// where the neighbours' positions come from.  The gathered x_j rows are the
// step's dominant traffic (every coupling reads x_j for every agent), and
// in the azimuth spin order consecutive rows share most of their
// neighbours.  So rows are taken in tiles of kTileRows consecutive rows:
// once per solve, tile_union lists each tile's distinct columns (its column
// union, at most kTileCols of them) and rewrites every coupling's column as
// its index in that list; each step, a workgroup (one tile, 64 agents)
// first copies x[union, its agents] into LDS -- one coalesced 256-byte read
// per column instead of one per coupling -- and its rows then gather from
// LDS.  Columns past kTileCols (a tile whose union is larger) are read from
// global memory as before.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sb_device.hpp"
#include "sb_kernels.hpp"

namespace sbt {

namespace {

constexpr int kT = 256;              // threads of the step workgroup (4 waves)
constexpr int kUnionCap = 4096;      // couplings of a tile tile_union sorts in LDS
constexpr uint16_t kGlobal = 0xFFFF; // "read this column from global memory"

template <bool NT, class T>
__device__ __forceinline__ T ld_nt(const T *p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <bool NT, class T>
__device__ __forceinline__ void st_nt(T v, T *p) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <int SEL>
__device__ __forceinline__ float fp8_to_f32(uint32_t word) {
    return __builtin_amdgcn_cvt_f32_fp8(static_cast<int>(word), SEL);
}

}  // namespace

// One workgroup per tile: sort the tile's padded columns (bitonic, in LDS),
// keep the distinct ones (the first kTileCols in ascending order go to
// tile_cols, their count to tile_u), and give every coupling of the tile
// the index of its column in that list, or kGlobal.
__global__ __launch_bounds__(kT) void tile_union(int n, const int *__restrict__ prow,
                                                 const int *__restrict__ pcol,
                                                 int *__restrict__ tile_cols, int *__restrict__ tile_u,
                                                 uint16_t *__restrict__ ploc) {
    __shared__ int s[kUnionCap];
    __shared__ int rank[kUnionCap];
    __shared__ int wsum[kT / 64];
    const int tt = blockIdx.x, t = threadIdx.x;
    const int i0 = tt * kTileRows, i1 = min(n, i0 + kTileRows);
    const int q0 = prow[i0], q1 = prow[i1];
    const int E = q1 - q0;
    if (E > kUnionCap) {  // too many couplings to sort here: all global
        for (int q = q0 + t; q < q1; q += kT) ploc[q] = kGlobal;
        if (t == 0) tile_u[tt] = 0;
        return;
    }
    int P = 1;
    while (P < E) P <<= 1;
    for (int k = t; k < P; k += kT) s[k] = k < E ? pcol[q0 + k] : INT32_MAX;
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int k = t; k < P; k += kT) {
                const int o = k ^ stride;
                if (o > k) {
                    const bool up = (k & size) == 0;
                    const int a = s[k], b = s[o];
                    if ((a > b) == up) {
                        s[k] = b;
                        s[o] = a;
                    }
                }
            }
            __syncthreads();
        }
    // distinct values: rank of the first occurrence of each (exclusive scan
    // of first-occurrence flags; each thread a contiguous run of entries)
    const int per = (E + kT - 1) / kT;
    const int k0 = min(E, t * per), k1 = min(E, k0 + per);
    int cnt = 0;
    for (int k = k0; k < k1; ++k) cnt += (k == 0 || s[k] != s[k - 1]) ? 1 : 0;
    int total = 0;
    int base = block_exclusive_scan(cnt, wsum, total);
    for (int k = k0; k < k1; ++k) {
        const bool first = k == 0 || s[k] != s[k - 1];
        rank[k] = base;  // for a first occurrence: its rank; otherwise unused
        if (first) {
            if (base < kTileCols) tile_cols[static_cast<size_t>(tt) * kTileCols + base] = s[k];
            ++base;
        }
    }
    if (t == 0) tile_u[tt] = min(total, kTileCols);
    __syncthreads();
    for (int q = q0 + t; q < q1; q += kT) {
        const int c = pcol[q];
        int lo = 0, hi = E;  // first position holding c
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (s[mid] < c) lo = mid + 1; else hi = mid;
        }
        const int r = rank[lo];
        ploc[q] = r < kTileCols ? static_cast<uint16_t>(r) : kGlobal;
    }
}

// One step: workgroup = (tile, 64 agents), lane = agent, each wave two rows.
template <int MODE, int JP, bool NT>
__global__ __launch_bounds__(kT) void sb_stream_tile(StreamArgs A, TileArgs T, int k,
                                                     const float *__restrict__ xin,
                                                     float *__restrict__ xout) {
    extern __shared__ float xs[];  // [kTileCols][64]
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int M = A.M;
    const int ntile = (A.n + kTileRows - 1) / kTileRows;
    const int nab = (M + 63) / 64;
    // XCD-contiguous: each XCD (workgroups dealt round robin) sweeps a
    // contiguous range of tiles of one agent block
    const int total = ntile * nab;
    const int per_xcd = (total + 7) / 8;
    const int v = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (v >= total) return;
    const int ab = v / ntile, tt = v % ntile;
    const int m = ab * 64 + lane;
    const bool live = m < M;
    const int ma = live ? m : 0;  // dead lanes read agent 0 (in bounds)
    const int U = T.tile_u[tt];
    const int *cols = T.tile_cols + static_cast<size_t>(tt) * kTileCols;
    for (int u = wave; u < U; u += kT / 64) {
        const int c = __builtin_amdgcn_readfirstlane(cols[u]);
        xs[u * 64 + lane] = xin[static_cast<size_t>(c) * M + ma];
    }
    __syncthreads();
    const float c0 = static_cast<float>(A.scal[0]);
    const float g = A.sched[k];
#pragma unroll
    for (int r = 0; r < kTileRows / (kT / 64); ++r) {
        const int i = tt * kTileRows + wave * (kTileRows / (kT / 64)) + r;
        if (i >= A.n) break;
        const float scale = JP == kJFp8 ? A.rowscale[i] : 1.0f;
        float acc = A.h[i];
        const int p1 = A.row_ptr[i + 1];
        for (int p = A.row_ptr[i]; p < p1; p += kStreamChunk) {
            const uint4 lw = *reinterpret_cast<const uint4 *>(T.ploc + p);  // 8 x uint16
            const uint32_t lp[4] = {lw.x, lw.y, lw.z, lw.w};
            float w[kStreamChunk];
            if constexpr (JP == kJFp8) {
                const uint2 codes = *reinterpret_cast<const uint2 *>(A.J8 + p);
                w[0] = scale * fp8_to_f32<0>(codes.x);
                w[1] = scale * fp8_to_f32<1>(codes.x);
                w[2] = scale * fp8_to_f32<2>(codes.x);
                w[3] = scale * fp8_to_f32<3>(codes.x);
                w[4] = scale * fp8_to_f32<0>(codes.y);
                w[5] = scale * fp8_to_f32<1>(codes.y);
                w[6] = scale * fp8_to_f32<2>(codes.y);
                w[7] = scale * fp8_to_f32<3>(codes.y);
            } else {
#pragma unroll
                for (int u = 0; u < kStreamChunk; ++u) w[u] = A.J[p + u];
            }
            float xv[kStreamChunk];
#pragma unroll
            for (int u = 0; u < kStreamChunk; ++u) {
                const uint32_t li = (lp[u >> 1] >> (16 * (u & 1))) & 0xFFFFu;
                if (li != kGlobal)
                    xv[u] = xs[li * 64 + lane];
                else
                    xv[u] = xin[static_cast<size_t>(A.col[p + u]) * M + ma];
            }
#pragma unroll
            for (int u = 0; u < kStreamChunk; ++u) acc = __builtin_fmaf(w[u], xv[u], acc);
        }
        if (live) {
            const size_t o = static_cast<size_t>(i) * M + m;
            float x = ld_nt<NT>(xin + o), y = ld_nt<NT>(A.y + o);
            sb_step<MODE>(x, y, acc, c0, g, A.dt, A.dta0);
            st_nt<NT>(x, xout + o);
            st_nt<NT>(y, A.y + o);
        }
    }
}

hipError_t launch_tile_union(int n, const int *prow, const int *pcol, const TileArgs &T,
                             hipStream_t st) {
    const int ntile = (n + kTileRows - 1) / kTileRows;
    tile_union<<<ntile, kT, 0, st>>>(n, prow, pcol, T.tile_cols, T.tile_u, T.ploc);
    return hipGetLastError();
}

template <int MODE, bool NT>
static hipError_t tile_step(int jprec, const StreamArgs &A, const TileArgs &T, int k,
                            const float *xin, float *xout, hipStream_t st) {
    const int ntile = (A.n + kTileRows - 1) / kTileRows;
    const int total = ntile * ((A.M + 63) / 64);
    const int grid = (total + 7) / 8 * 8;
    const size_t lds = sizeof(float) * kTileCols * 64;
    if (jprec == kJFp8)
        return launch_with_lds(sb_stream_tile<MODE, kJFp8, NT>, dim3(grid), dim3(kT), lds, st, A, T, k,
                               xin, xout);
    if (jprec != kJFp32) return hipErrorInvalidValue;  // FP32 or per-row FP8 only
    return launch_with_lds(sb_stream_tile<MODE, kJFp32, NT>, dim3(grid), dim3(kT), lds, st, A, T, k,
                           xin, xout);
}

hipError_t launch_stream_tile(int mode, int jprec, const StreamArgs &A, const TileArgs &T, int k,
                              const float *xin, float *xout, hipStream_t st) {
    // own-row x, y streamed past the caches when the state exceeds the
    // Infinity Cache, as in sb_stream
    const bool nt = static_cast<size_t>(A.n) * A.M * sizeof(float) * 3 > (size_t(256) << 20);
    if (mode == kASB)
        return nt ? tile_step<kASB, true>(jprec, A, T, k, xin, xout, st)
                  : tile_step<kASB, false>(jprec, A, T, k, xin, xout, st);
    return nt ? tile_step<kBSB, true>(jprec, A, T, k, xin, xout, st)
              : tile_step<kBSB, false>(jprec, A, T, k, xin, xout, st);
}

}  // namespace sbt
