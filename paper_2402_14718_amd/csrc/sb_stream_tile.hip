// Streaming bSB / aSB step with each row tile's neighbour positions staged
// in LDS (gfx950).
//
// Same step as sb_stream_v4 (paper section "Simulated Bifurcation", Eq. 5-8
// and Eq. 1-4): one launch per step, the coupling sum of each row seeded
// with h_i and taken over its padded CSR row in order, the fused update of
// sb_device.hpp -- so the results are bit-identical to it.  What differs is
// where the neighbours' positions come from.  Every coupling reads x_j for
// every agent, and those gathers are the step's dominant traffic through the
// vector-memory path; in the azimuth spin order consecutive rows share
// neighbours.  So, once per solve, tile_plan cuts the rows into tiles:
// super tiles of kTileSuper consecutive rows, each cut greedily into runs of
// consecutive rows whose column union (the distinct columns of their padded
// rows) has at most `ucap` entries.  It stores each tile's union, ascending,
// and rewrites every coupling's column as its index in that list.  Each
// step, a workgroup (one super tile, 64 agents) takes its tiles in turn:
// it copies x[union, its agents] into LDS -- one 256-byte read per distinct
// column instead of one per coupling, all of a tile's reads in flight
// together -- and its four waves then run the tile's rows from LDS.  A row
// longer than ucap is a tile of its own that reads global memory.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sb_device.hpp"
#include "sb_kernels.hpp"
#include "sb_stream_kernels.hpp"
#include "sb_stream_chunk.hpp"

namespace sbt {

namespace {

constexpr int kT = 256;              // threads of the plan and step workgroups (4 waves)
constexpr int kStage = 8;            // 16-byte staging loads in flight per thread
static_assert(kTileColsMax <= kT, "tile_plan gives one thread to each entry of a row");
static_assert(kTileNnz >= kTileColsMax, "a row that fits the columns fits the couplings");

__device__ __forceinline__ int lower_bound(const int *v, int len, int c) {
    int lo = 0, hi = len;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (v[mid] < c)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Bitonic sort of v[0..P) ascending, P a power of two <= kT.
__device__ void bitonic_sort(int *v, int P) {
    const int t = threadIdx.x;
    for (int size = 2; size <= P; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            if (t < P) {
                const int o = t ^ stride;
                if (o > t) {
                    const bool up = (t & size) == 0;
                    const int a = v[t], b = v[o];
                    if ((a > b) == up) {
                        v[t] = b;
                        v[o] = a;
                    }
                }
            }
            __syncthreads();
        }
}

}  // namespace

// One workgroup per super tile.  The tile being built keeps its column
// union sorted in LDS; each next row's distinct columns not yet in it are
// counted (its padded columns sorted, first occurrences looked up in the
// union) and merged in, unless that would pass ucap columns or kTileNnz
// padded couplings, which closes the tile.
// Closing writes the union to tile_cols from the tile's first padded
// coupling on (a union is never longer than its rows' padded couplings),
// each coupling's index in it to ploc, and (first row, union size) to
// tile_info.
__global__ __launch_bounds__(kT) void tile_plan(int n, const int *__restrict__ prow,
                                                const int *__restrict__ pcol, TileArgs T) {
    __shared__ int set_a[kTileColsMax], set_b[kTileColsMax];
    __shared__ int row[kTileColsMax];
    __shared__ int fresh[kTileColsMax];
    __shared__ int wsum[kT / 64];
    const int s = blockIdx.x, t = threadIdx.x;
    const int ucap = T.ucap;
    const int r0 = s * kTileSuper, r1 = min(n, r0 + kTileSuper);
    int *cur = set_a, *nxt = set_b;
    int U = 0, first = r0, nt = 0, nnz = 0;  // the open tile: union size, padded couplings
    auto close = [&](int end) {
        const int base = prow[first];
        for (int u = t; u < U; u += kT) T.tile_cols[base + u] = cur[u];
        for (int q = base + t; q < prow[end]; q += kT)
            T.ploc[q] = U > 0 ? static_cast<uint16_t>(lower_bound(cur, U, pcol[q])) : kTileGlobal;
        if (t == 0) T.tile_info[s * kTileSuper + nt] = make_int2(first, U);
        ++nt;
        first = end;
        U = 0;
        nnz = 0;
        __syncthreads();
    };
    // distinct columns of the sorted row absent from the union -> fresh
    auto count_new = [&](int L) {
        int f = 0;
        if (t < L) {
            const int c = row[t];
            const bool first_occ = t == 0 || row[t - 1] != c;
            const int at = lower_bound(cur, U, c);
            f = first_occ && !(at < U && cur[at] == c);
        }
        int total = 0;
        const int pos = block_exclusive_scan(f, wsum, total);
        if (f) fresh[pos] = row[t];
        __syncthreads();
        return total;
    };
    for (int r = r0; r < r1; ++r) {
        const int q0 = prow[r], L = prow[r + 1] - q0;
        if (L > ucap) {  // longer than a tile holds: a tile of its own, from global memory
            if (r > first) close(r);
            close(r + 1);
            continue;
        }
        int P = 1;
        while (P < L) P <<= 1;
        if (t < P) row[t] = t < L ? pcol[q0 + t] : INT32_MAX;
        __syncthreads();
        bitonic_sort(row, P);
        int cnt = count_new(L);
        if (U + cnt > ucap || nnz + L > kTileNnz) {
            close(r);
            cnt = count_new(L);
        }
        nnz += L;
        // merge: an entry's place is its index plus how many of the other
        // list precede it (the lists are disjoint)
        for (int u = t; u < U; u += kT) nxt[u + lower_bound(fresh, cnt, cur[u])] = cur[u];
        for (int j = t; j < cnt; j += kT) nxt[j + lower_bound(cur, U, fresh[j])] = fresh[j];
        __syncthreads();
        int *tmp = cur;
        cur = nxt;
        nxt = tmp;
        U += cnt;
    }
    if (first < r1) close(r1);
    if (t == 0) T.tile_n[s] = nt;
}

// A coupling decoded to FP32 as the streaming step uses it, except that
// the per-row FP8 form leaves out the row's scale (applied at use, the same
// product as the untiled step's).
template <int JP>
__device__ __forceinline__ float coupling_value(const StreamArgs &A, int q) {
    if constexpr (JP == kJFp8)
        return e4m3_to_f32<0>(A.J8[q]);
    else if constexpr (JP == kJFp8Blk)
        return A.blkscale[q / kStreamChunk] * e4m3_to_f32<0>(A.J8[q]);
    else if constexpr (JP == kJBf16x2)
        return bf16x2_value(A.J2[q]);
    else
        return A.J[q];
}

// One step: workgroup = (super tile, 64 agents), lane = agent; the tiles of
// the super tile in turn.  Staging puts the tile's union positions and its
// couplings (value, index in the union) in LDS with every load of a batch
// in flight at once; the four waves then take the tile's rows round robin.
// A row's couplings are read 64 at a time, one per lane, and handed to the
// whole wave in CSR order by lane reads, so the loop over a row's couplings
// waits only on LDS.  V4: M % 4 == 0, positions staged 16 bytes (4 agents)
// per load.  The arrays come in as separate non-aliasing arguments (read
// only, except x out and y).
template <int MODE, int JP, bool NT, bool V4>
__global__ __launch_bounds__(kT) void sb_stream_tile(
    StreamArgs A, int ucap, int k, const int *__restrict__ row_ptr, const int *__restrict__ col,
    const float *__restrict__ Jf, const uint8_t *__restrict__ J8, const float *__restrict__ rowscale,
    const float *__restrict__ blkscale, const uint32_t *__restrict__ J2, const float *__restrict__ h,
    const int2 *__restrict__ tinfo, const int *__restrict__ tn, const int *__restrict__ tcols,
    const uint16_t *__restrict__ ploc, const float *__restrict__ xin, float *__restrict__ xout,
    float *__restrict__ y) {
    extern __shared__ float xs[];  // [ucap][64] positions, then couplings
    float *cj = xs + 64 * ucap;                                 // [kTileNnz] values
    uint16_t *cl = reinterpret_cast<uint16_t *>(cj + kTileNnz);  // [kTileNnz] union indices
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, t = threadIdx.x;
    const int M = A.M;
    StreamArgs C = A;  // the coupling arrays, as the restrict arguments
    C.J = Jf;
    C.J8 = J8;
    C.blkscale = blkscale;
    C.J2 = J2;
    const int nsuper = (A.n + kTileSuper - 1) / kTileSuper;
    const int nab = (M + 63) / 64;
    // XCD-contiguous: each XCD (workgroups are dealt round robin) sweeps a
    // contiguous range of super tiles of one agent block
    const int total = nsuper * nab;
    const int per_xcd = (total + 7) / 8;
    const int v = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (v >= total) return;
    const int ab = v / nsuper, s = v % nsuper;
    const int m = ab * 64 + lane;
    const bool live = m < M;
    const int ma = live ? m : 0;  // dead lanes read agent 0 (in bounds)
    const int r1 = min(A.n, (s + 1) * kTileSuper);
    const int ntile = tn[s];
    const int lmax = ucap - 1;
    const float c0 = static_cast<float>(A.scal[0]);
    const float g = A.sched[k];
    for (int tt = 0; tt < ntile; ++tt) {
        const int2 info = tinfo[s * kTileSuper + tt];
        const int first = __builtin_amdgcn_readfirstlane(info.x);
        const int U = __builtin_amdgcn_readfirstlane(info.y);
        const int last = __builtin_amdgcn_readfirstlane(
            tt + 1 < ntile ? tinfo[s * kTileSuper + tt + 1].x : r1);
        const int base = __builtin_amdgcn_readfirstlane(row_ptr[first]);
        const int *cols = tcols + base;
        if (tt > 0) __syncthreads();  // the previous tile's rows are done with LDS
        if (U > 0) {
            // couplings: at most kTileNnz (the plan's bound), four per thread
            const int nc = row_ptr[last] - base;
#pragma unroll
            for (int j = 0; j < kTileNnz / kT + 1; ++j) {
                const int e = j * kT + t;
                if (e < nc) {
                    cj[e] = coupling_value<JP>(C, base + e);
                    cl[e] = ploc[base + e];
                }
            }
            // positions: the column indices of kStage entries, then their
            // positions, then the LDS stores (entries past the union re-read
            // its last column and are not stored; dead agents are stored as 0)
            constexpr int kPer = V4 ? 16 : 64;  // staging entries per column
            const int ne = U * kPer;
            for (int b = 0; b < ne; b += kT * kStage) {
                int ci[kStage];
#pragma unroll
                for (int j = 0; j < kStage; ++j)
                    ci[j] = cols[static_cast<unsigned>(min(b + j * kT + t, ne - 1)) / kPer];
                if constexpr (V4) {
                    float4 st[kStage];
#pragma unroll
                    for (int j = 0; j < kStage; ++j) {
                        const int a = ab * 64 + ((b + j * kT + t) & 15) * 4;
                        st[j] = *reinterpret_cast<const float4 *>(xin + static_cast<size_t>(ci[j]) * M +
                                                                  (a < M ? a : 0));
                    }
#pragma unroll
                    for (int j = 0; j < kStage; ++j) {
                        const int idx = b + j * kT + t;
                        const bool dead = ab * 64 + (idx & 15) * 4 >= M;
                        if (idx < ne)
                            reinterpret_cast<float4 *>(xs)[idx] =
                                dead ? make_float4(0.0f, 0.0f, 0.0f, 0.0f) : st[j];
                    }
                } else {
                    float st[kStage];
#pragma unroll
                    for (int j = 0; j < kStage; ++j) {
                        const int a = ab * 64 + ((b + j * kT + t) & 63);
                        st[j] = xin[static_cast<size_t>(ci[j]) * M + (a < M ? a : 0)];
                    }
#pragma unroll
                    for (int j = 0; j < kStage; ++j) {
                        const int idx = b + j * kT + t;
                        if (idx < ne) xs[idx] = ab * 64 + (idx & 63) < M ? st[j] : 0.0f;
                    }
                }
            }
            __syncthreads();
        }
        for (int i = first + wave; i < last; i += kT / 64) {
            const float scale = JP == kJFp8 ? rowscale[i] : 1.0f;
            float acc = h[i];
            const int p0 = row_ptr[i], p1 = row_ptr[i + 1];
            // the row's own x, y in flight during its coupling sum
            const size_t o = static_cast<size_t>(i) * M + ma;
            float x = ld_stream<NT>(xin + o), yv = ld_stream<NT>(y + o);
            if (U > 0) {
                for (int pb = p0 - base; pb < p1 - base; pb += 64) {
                    const int e = min(pb + lane, p1 - base - 1);
                    const int vl = min(static_cast<int>(cl[e]), lmax);
                    float vj = cj[e];
                    if constexpr (JP == kJFp8) vj = scale * vj;
                    const int cnt = min(64, p1 - base - pb);  // a multiple of kStreamChunk
                    for (int u = 0; u < cnt; u += kStreamChunk) {
                        float xv[kStreamChunk];
#pragma unroll
                        for (int c = 0; c < kStreamChunk; ++c)
                            xv[c] = xs[__builtin_amdgcn_readlane(vl, u + c) * 64 + lane];
#pragma unroll
                        for (int c = 0; c < kStreamChunk; ++c)
                            acc = __builtin_fmaf(
                                __int_as_float(__builtin_amdgcn_readlane(__float_as_int(vj), u + c)),
                                xv[c], acc);
                    }
                }
            } else {
                for (int p = p0; p < p1; p += kStreamChunk) {
                    const int4 ca = *reinterpret_cast<const int4 *>(col + p);
                    const int4 cb = *reinterpret_cast<const int4 *>(col + p + 4);
                    const int c[kStreamChunk] = {ca.x, ca.y, ca.z, ca.w, cb.x, cb.y, cb.z, cb.w};
                    float w[kStreamChunk];
                    load_chunk<JP>(C, p, scale, w);
                    float xv[kStreamChunk];
#pragma unroll
                    for (int u = 0; u < kStreamChunk; ++u) xv[u] = xin[static_cast<size_t>(c[u]) * M + ma];
#pragma unroll
                    for (int u = 0; u < kStreamChunk; ++u) acc = __builtin_fmaf(w[u], xv[u], acc);
                }
            }
            if (live) {
                if constexpr (MODE == kASB)
                    sb_update_asb(x, yv, acc, c0, g, A.dt, A.dta0);
                else
                    sb_update(x, yv, acc, c0, g, A.dt, A.dta0);
                st_stream<NT>(x, xout + o);
                st_stream<NT>(yv, y + o);
            }
        }
    }
}

hipError_t launch_tile_plan(int n, const int *prow, const int *pcol, const TileArgs &T,
                            hipStream_t st) {
    if (T.ucap < kStreamChunk || T.ucap > kTileColsMax) return hipErrorInvalidValue;
    const int nsuper = (n + kTileSuper - 1) / kTileSuper;
    tile_plan<<<nsuper, kT, 0, st>>>(n, prow, pcol, T);
    return hipGetLastError();
}

namespace {

template <int MODE, bool NT, bool V4>
hipError_t tile_step(int jprec, const StreamArgs &A, const TileArgs &T, int k, const float *xin,
                     float *xout, hipStream_t st) {
    const int nsuper = (A.n + kTileSuper - 1) / kTileSuper;
    const int total = nsuper * ((A.M + 63) / 64);
    const dim3 grid((total + 7) / 8 * 8);
    const size_t lds = tile_lds_bytes(T.ucap);
    auto go = [&](auto kern) {
        return launch_with_lds(kern, grid, dim3(kT), lds, st, A, T.ucap, k, A.row_ptr, A.col, A.J,
                               A.J8, A.rowscale, A.blkscale, A.J2, A.h,
                               static_cast<const int2 *>(T.tile_info),
                               static_cast<const int *>(T.tile_n),
                               static_cast<const int *>(T.tile_cols),
                               static_cast<const uint16_t *>(T.ploc), xin, xout, A.y);
    };
    switch (jprec) {
        case kJFp8: return go(sb_stream_tile<MODE, kJFp8, NT, V4>);
        case kJFp8Blk: return go(sb_stream_tile<MODE, kJFp8Blk, NT, V4>);
        case kJBf16x2: return go(sb_stream_tile<MODE, kJBf16x2, NT, V4>);
        case kJFp32: return go(sb_stream_tile<MODE, kJFp32, NT, V4>);
        default: return hipErrorInvalidValue;
    }
}

template <int MODE>
hipError_t tile_step_mode(bool nt, int jprec, const StreamArgs &A, const TileArgs &T, int k,
                          const float *xin, float *xout, hipStream_t st) {
    const bool v4 = A.M % 4 == 0;
    if (nt)
        return v4 ? tile_step<MODE, true, true>(jprec, A, T, k, xin, xout, st)
                  : tile_step<MODE, true, false>(jprec, A, T, k, xin, xout, st);
    return v4 ? tile_step<MODE, false, true>(jprec, A, T, k, xin, xout, st)
              : tile_step<MODE, false, false>(jprec, A, T, k, xin, xout, st);
}

}  // namespace

hipError_t launch_stream_tile(int mode, int jprec, const StreamArgs &A, const TileArgs &T, int k,
                              const float *xin, float *xout, hipStream_t st) {
    if (T.ucap < kStreamChunk || T.ucap > kTileColsMax) return hipErrorInvalidValue;
    // own-row x, y streamed past the caches when the state exceeds the
    // Infinity Cache, as in sb_stream
    const bool nt = static_cast<size_t>(A.n) * A.M * sizeof(float) * 3 > (size_t(256) << 20);
    if (mode == kASB) return tile_step_mode<kASB>(nt, jprec, A, T, k, xin, xout, st);
    if (mode == kBSB) return tile_step_mode<kBSB>(nt, jprec, A, T, k, xin, xout, st);
    return hipErrorInvalidValue;
}

}  // namespace sbt
