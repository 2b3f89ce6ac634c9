// dSB streaming step on the matrix cores (gfx950).
//
// Paper section "Simulated Bifurcation", Eq. 9-12: the dSB coupling term
// of row i for agent a is h_i + sum_j J_ij sgn(x_j(a)).  Over a block of
// 16 consecutive rows, the listed columns of the block and a group of 16
// agents, that sum is a matrix product: couplings (16 rows x listed
// columns) times signs (listed columns x 16 agents).  sgn(x) = +-1 is exact
// in any operand type, so with couplings whose stored form is itself an
// operand type the products are exact and only the order of the FP32
// additions differs from the CSR step:
//   FP8 (e4m3, one scale per row): the codes are the operand and the row's
//     scale multiplies the row's sum once, F_i = h_i + s_i sum_j q_ij sgn_j;
//   BF16 hi + lo: two products on the same signs, F_i = h_i + sum hi sgn +
//     sum lo sgn;
//   FP32: each coupling split exactly into three BF16 terms (8 significant
//     bits each), three products on the same signs; FP8 with a scale per
//     block of 8 couplings: the FP32 value scale x code, split the same way;
//   BF16 or FP16 (the FP32 coupling rounded once): one product.
// The positions x and momenta y update in place as in the CSR step
// (sb_update); the signs live in this step's own records (16 bytes per row
// and group of 128 agents, bit t of byte c = agent 16 t + c of the group).
//
// In the azimuth spin order the couplings fill about 0.16 of a block's
// rows x listed columns on the stress event and 0.09 on the sparse events,
// so the matrix cores do 6-11 x the arithmetic of the couplings themselves,
// cheaply; what a K-step costs is one sign byte per listed column and lane
// and a few shifts per tile to spread it into the +-1 operand.
//
// One wave = one block x one group of 128 agents (8 tiles of 16).  Per
// K-step of 32 listed columns lane (g = lane / 16, c = lane % 16) holds,
// for each tile t, the signs of agent 16 t + c on listed columns 8 g ..
// 8 g + 7 (bit t of the lane's 8 sign bytes; the first operand, agents x
// columns) and row c's couplings on the same columns (the second operand,
// columns x rows), so the instruction pairs them; the 16 x 16 result of
// tile t (agents x rows) holds, in lane (g, c), agents 16 t + 4 g .. + 3 of
// row c: four consecutive agents, one 16-byte access of x and of y, and
// the lane's 32 new signs of row c are dword g of the row's record.  x and
// y are kept in this step's own tiled layout (mfma_state_floats), where a
// wave's accesses for one t are one contiguous 1 KB run: in the spin-major
// layout they touch 16 rows x 64 bytes and the step ran 1.4 x slower.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sb_device.hpp"
#include "sb_kernels.hpp"
#include "sb_stream_kernels.hpp"
#include "sb_stream_chunk.hpp"
#include "sb_stream_mfma.hpp"

namespace sbt {

namespace {

constexpr int kBR = kMfmaRows;
constexpr int kBK = kMfmaK;
constexpr int kChunkSteps = 4;   // K-steps whose sign records are staged in LDS at once
constexpr int kScanThreads = 1024;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Walks the union of block b's rows (padded CSR; a row's own column marks
// its padding) in ascending column order, calling f(column, at[kBR]) with
// at[r] the row's entry for that column or -1.
template <class F>
__device__ __forceinline__ void block_union(int n, const int *prow, const int *pcol, int b, F &&f) {
    int pos[kBR], end[kBR], head[kBR];  // head: the row's next column (INT32_MAX: none)
#pragma unroll
    for (int r = 0; r < kBR; ++r) {
        const int i = b * kBR + r;
        pos[r] = i < n ? prow[i] : 0;
        end[r] = i < n ? prow[i + 1] : 0;
        while (pos[r] < end[r] && pcol[end[r] - 1] == i) --end[r];  // drop the padding
        head[r] = pos[r] < end[r] ? pcol[pos[r]] : INT32_MAX;
    }
    while (true) {
        int c = INT32_MAX;
#pragma unroll
        for (int r = 0; r < kBR; ++r) c = min(c, head[r]);
        if (c == INT32_MAX) break;
        int at[kBR];
#pragma unroll
        for (int r = 0; r < kBR; ++r) {
            at[r] = -1;
            if (head[r] == c) {
                at[r] = pos[r]++;
                head[r] = pos[r] < end[r] ? pcol[pos[r]] : INT32_MAX;
            }
        }
        f(c, at);
    }
}

__global__ __launch_bounds__(256) void mfma_count(int n, int nb, const int *__restrict__ prow,
                                                  const int *__restrict__ pcol, int *__restrict__ cnt) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= nb) return;
    int d = 0;
    block_union(n, prow, pcol, b, [&](int, const int *) { ++d; });
    cnt[b] = (d + kBK - 1) / kBK;
}

// cnt[0..nb) -> off[0..nb] (exclusive prefix sums, off[nb] = total); one
// workgroup, each thread a contiguous range.
__global__ __launch_bounds__(kScanThreads) void mfma_scan(int nb, const int *__restrict__ cnt,
                                                          int *__restrict__ off) {
    __shared__ int tot[kScanThreads];
    const int t = threadIdx.x;
    const int per = (nb + kScanThreads - 1) / kScanThreads;
    const int b0 = min(nb, t * per), b1 = min(nb, b0 + per);
    int sum = 0;
    for (int b = b0; b < b1; ++b) sum += cnt[b];
    tot[t] = sum;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {
        const int v = t >= d ? tot[t - d] : 0;
        __syncthreads();
        tot[t] += v;
        __syncthreads();
    }
    int at = tot[t] - sum;
    for (int b = b0; b < b1; ++b) {
        off[b] = at;
        at += cnt[b];
    }
    if (t == kScanThreads - 1) off[nb] = tot[t];
}

// FP32 -> BF16, round to nearest even (finite values).
__device__ __forceinline__ uint32_t bf16_bits(float v) {
    const uint32_t u = __float_as_uint(v);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// An FP32 coupling as BF16 terms hi + mid + lo, exactly: each residual is
// exact in FP32 (Sterbenz), the last one has at most 8 significant bits.
__device__ __forceinline__ void bf16_triple(float v, uint32_t (&t)[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        t[k] = bf16_bits(v);
        v -= __uint_as_float(t[k] << 16);
    }
}

// Lists block b's columns and writes every operand word of its K-steps:
// listed column u (0-based in the block) of row r is element u % 8 of lane
// 16 ((u % 32) / 8) + r in K-step u / 32 (FP8: byte e of the lane's word;
// BF16 terms: term k in words 2 k and 2 k + 1, 16 bits per element); zeros
// where a row has no coupling and in the padding, whose column repeats the
// last listed one.  A lane's word is assembled over 8 consecutive listed
// columns and stored whole.
template <int JP>
__global__ __launch_bounds__(256) void mfma_fill(int nb, StreamArgs A, const int *__restrict__ koff,
                                                 int *__restrict__ kcol, uint64_t *__restrict__ kA) {
    constexpr int W = mfma_words(JP);
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= nb) return;
    const int ks0 = koff[b], u1 = (koff[b + 1] - ks0) * kBK;
    uint64_t buf[kBR][W];
#pragma unroll
    for (int r = 0; r < kBR; ++r)
#pragma unroll
        for (int w = 0; w < W; ++w) buf[r][w] = 0;
    auto flush = [&](int u) {  // u: the last listed column of a group of 8
        const size_t lane0 = static_cast<size_t>(ks0 + u / kBK) * 64 + 16 * ((u % kBK) / 8);
#pragma unroll
        for (int r = 0; r < kBR; ++r)
#pragma unroll
            for (int w = 0; w < W; ++w) {
                kA[(lane0 + r) * W + w] = buf[r][w];
                buf[r][w] = 0;
            }
    };
    int u = 0, last = 0;
    block_union(A.n, A.row_ptr, A.col, b, [&](int c, const int *at) {
        kcol[static_cast<size_t>(ks0) * kBK + u] = c;
        const int e = u % 8;
#pragma unroll
        for (int r = 0; r < kBR; ++r) {
            if (at[r] < 0) continue;
            if constexpr (JP != kJFp8) {
                uint32_t term[3] = {0u, 0u, 0u};
                if constexpr (JP == kJBf16) {
                    term[0] = bf16_bits(A.J[at[r]]);
                } else if constexpr (JP == kJFp16) {
                    term[0] = __builtin_bit_cast(uint16_t, static_cast<_Float16>(A.J[at[r]]));
                } else if constexpr (JP == kJBf16x2) {
                    term[0] = A.J2[at[r]] >> 16;
                    term[1] = A.J2[at[r]] & 0xFFFFu;
                } else if constexpr (JP == kJFp8Blk) {  // the CSR step's decoded value
                    bf16_triple(A.blkscale[at[r] / kStreamChunk] * e4m3_to_f32<0>(A.J8[at[r]]), term);
                } else {
                    bf16_triple(A.J[at[r]], term);
                }
                const int sh = 16 * (e % 4);
#pragma unroll
                for (int k = 0; k < W / 2; ++k)
#pragma unroll
                    for (int w = 0; w < 2; ++w)
                        if (e / 4 == w) buf[r][2 * k + w] |= static_cast<uint64_t>(term[k]) << sh;
            } else {
                buf[r][0] |= static_cast<uint64_t>(A.J8[at[r]]) << (8 * e);
            }
        }
        last = c;
        if (e == 7) flush(u);
        ++u;
    });
    for (; u < u1; ++u) {
        kcol[static_cast<size_t>(ks0) * kBK + u] = last;
        if (u % 8 == 7) flush(u);
    }
}

// Workgroup id -> (group of 4 blocks, agent group), XCD-contiguous: each
// XCD sweeps one contiguous range of blocks, all agent groups of a block
// next to each other, so the block's operand tiles and listed columns are
// reused from that XCD's L2 and the sign records its blocks read (all
// agent groups of a column share a line) stay there.
__device__ __forceinline__ bool mfma_block(int ngb, int nab, int &gb, int &ab) {
    const int total = ngb * nab;
    const int per_xcd = (total + 7) / 8;
    const int v = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (v >= total) return false;
    ab = v % nab;
    gb = v / nab;
    return true;
}

// Sign records from the current positions (layout of mfma_sign_bytes).
__global__ __launch_bounds__(256) void mfma_signs(int n, int M, const float *__restrict__ x,
                                                  uint8_t *__restrict__ S) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;  // (row, group, c)
    const int R = mfma_groups(M);
    if (idx >= static_cast<int64_t>(n) * R * 16) return;
    const int i = static_cast<int>(idx / (R * 16));
    const int grp = static_cast<int>(idx / 16 % R), c = static_cast<int>(idx % 16);
    uint32_t byte = 0;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int m = kMfmaGroup * grp + 16 * t + c;
        if (m < M && x[static_cast<size_t>(i) * M + m] >= 0.0f) byte |= 1u << t;
    }
    S[idx] = static_cast<uint8_t>(byte);
}

// Spin-major x[i M + m] <-> the step's tiles (layout of mfma_state_floats);
// one thread per 16-byte run of a tile.
__global__ __launch_bounds__(256) void mfma_state(int n, int M, bool to_tiles, const float *__restrict__ src,
                                                  float *__restrict__ dst) {
    const int R = mfma_groups(M);
    const int64_t q = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (q >= static_cast<int64_t>(mfma_state_floats(n, M) / 4)) return;
    const int64_t tile = q / 512;
    const int w = static_cast<int>(q % 512), t = w / 64, lane = w % 64;
    const int b = static_cast<int>(tile / R), ab = static_cast<int>(tile % R);
    const int i = b * kBR + (lane & 15), m = kMfmaGroup * ab + 16 * t + 4 * (lane >> 4);
    const size_t row = static_cast<size_t>(i) * M;
    if (to_tiles) {
        f32x4 v = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (i < n && m + r < M) v[r] = src[row + m + r];
        *reinterpret_cast<f32x4 *>(dst + 4 * q) = v;
    } else if (i < n) {
        const f32x4 v = *reinterpret_cast<const f32x4 *>(src + 4 * q);
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (m + r < M) dst[row + m + r] = v[r];
    }
}

}  // namespace

// One dSB step: a wave = one block of 16 rows x one group of 128 agents.
template <int JP, bool NT>
__global__ __launch_bounds__(256) void sb_stream_mfma(StreamArgs A, int k, const int *__restrict__ koff,
                                                      const int *__restrict__ kcol,
                                                      const uint64_t *__restrict__ kA,
                                                      const float *__restrict__ h,
                                                      const float *__restrict__ rowscale,
                                                      float *__restrict__ x, float *__restrict__ y,
                                                      const uint8_t *__restrict__ Sin,
                                                      uint8_t *__restrict__ Sout) {
    constexpr int T = kMfmaGroup / 16;    // tiles of 16 agents
    constexpr int W = mfma_words(JP);     // operand words per lane and K-step
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int M = A.M, R = mfma_groups(M);
    const int nb = (A.n + kBR - 1) / kBR;
    // When the state streams from HBM (NT), operands wider than one word per
    // lane (the 16-bit forms) are shared: a workgroup takes one block and up
    // to four agent groups (one per wave) and stages each chunk's operand
    // tiles in LDS once for all of them (measured on the stress event: BF16
    // pairs 0.452 -> 0.400 ms, FP32 0.490 -> 0.434).  Otherwise workgroups
    // take four blocks of one agent group, with no barriers and a third wave
    // per SIMD (cache-resident precision event, FP32: 23.6 against 27.8 us
    // with sharing).
    constexpr bool kShare = W > 1 && NT;
    int b, ab;
    bool active = true;   // the wave has an agent group (shared form: ab < R)
    if constexpr (kShare) {
        int ac;
        if (!mfma_block(nb, (R + 3) / 4, b, ac)) return;
        b = __builtin_amdgcn_readfirstlane(b);
        ab = __builtin_amdgcn_readfirstlane(ac * 4 + wave);
        active = ab < R;
    } else {
        int gb;
        if (!mfma_block((nb + 3) / 4, R, gb, ab)) return;
        b = __builtin_amdgcn_readfirstlane(gb * 4 + wave);
        if (b >= nb) return;
    }
    const int g = lane >> 4, c = lane & 15;
    f32x4 acc[T];
#pragma unroll
    for (int t = 0; t < T; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    // The lane's x, y (row 16 b + c, agents 128 ab + 16 t + 4 g + r: 16
    // bytes at tile + 256 t, padding included) are loaded before the
    // coupling sums, so their latency hides behind them.
    const size_t tile = (static_cast<size_t>(b) * R + ab) * (kBR * kMfmaGroup) + 4 * lane;
    f32x4 xp[T], yp[T];
    if (active) {
#pragma unroll
        for (int t = 0; t < T; ++t) {
            xp[t] = ld_stream<NT>(reinterpret_cast<const f32x4 *>(x + tile + 256 * t));
            yp[t] = ld_stream<NT>(reinterpret_cast<const f32x4 *>(y + tile + 256 * t));
        }
    }

    // The block's sign records pass through LDS, kChunkSteps K-steps at a
    // time: each lane fetches two listed columns' whole 16-byte records
    // (two loads instead of eight per K-step on the texture path, whose
    // cost is per instruction), and the K-steps read their sign bytes from
    // LDS.  A 16-byte pad after every 8 slots puts the four lane groups'
    // records on different banks.  Columns are fetched two chunks ahead,
    // records one chunk ahead; FP8 operands one K-step ahead, shared
    // operands one chunk ahead (wave w fetches K-step w of the chunk).
    constexpr int kSlots = kChunkSteps * kBK;
    __shared__ uint4 rec_lds[4][kSlots + kSlots / 8];
    uint4 *lds = rec_lds[wave];
    const int ks0 = koff[b], ks1 = koff[b + 1];
    const int nk = ks1 - ks0, nch = (nk + kChunkSteps - 1) / kChunkSteps;
    int cn[2];
    uint4 rn[2];
    uint64_t an[W];
    __shared__ uint64_t op_lds[kShare ? kChunkSteps * 64 * W : 1];
    auto load_cols = [&](int j) {
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            const int u = j * kSlots + lane + 64 * hh;  // block-relative listed column
            cn[hh] = u < nk * kBK ? kcol[static_cast<size_t>(ks0) * kBK + u] : -1;
        }
    };
    auto load_recs = [&]() {
#pragma unroll
        for (int hh = 0; hh < 2; ++hh)
            rn[hh] = cn[hh] >= 0
                         ? *reinterpret_cast<const uint4 *>(Sin + (static_cast<size_t>(cn[hh]) * R + ab) * 16)
                         : uint4{0u, 0u, 0u, 0u};
    };
    auto load_operand = [&](int ks) {
#pragma unroll
        for (int w = 0; w < W; ++w) an[w] = kA[(static_cast<size_t>(ks) * 64 + lane) * W + w];
    };
    // shared forms: this wave's K-step of chunk j (kept in `an` until stored)
    auto load_chunk_operand = [&](int j) {
        if (j * kChunkSteps + wave < nk) load_operand(ks0 + j * kChunkSteps + wave);
    };
    if (nch > 0) {
        if (active) {
            load_cols(0);
            load_recs();
            if (nch > 1) load_cols(1);
        }
        if constexpr (kShare)
            load_chunk_operand(0);
        else
            load_operand(ks0);
    }
    for (int j = 0; j < nch; ++j) {
        __builtin_amdgcn_wave_barrier();    // the previous chunk's LDS reads come first
        if (active) {
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                const int sl = lane + 64 * hh;
                lds[sl + sl / 8] = rn[hh];
            }
        }
        if constexpr (kShare) {
            __syncthreads();                // every wave is done with the previous chunk's operands
            if (j * kChunkSteps + wave < nk) {
#pragma unroll
                for (int w = 0; w < W; ++w) op_lds[(wave * 64 + lane) * W + w] = an[w];
            }
            __syncthreads();
        }
        __builtin_amdgcn_wave_barrier();
        if (j + 1 < nch) {
            if (active) {
                load_recs();
                if (j + 2 < nch) load_cols(j + 2);
            }
            if constexpr (kShare) load_chunk_operand(j + 1);
        }
        if (!active) continue;
        const int kend = min(kChunkSteps, nk - j * kChunkSteps);
        for (int kk = 0; kk < kend; ++kk) {
            const int ks = ks0 + j * kChunkSteps + kk;
            uint32_t s8[8];
            uint64_t a8[W];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int sl = kk * kBK + 8 * g + e;
                s8[e] = reinterpret_cast<const uint8_t *>(lds + sl + sl / 8)[c];
            }
            if constexpr (kShare) {
#pragma unroll
                for (int w = 0; w < W; ++w) a8[w] = op_lds[(kk * 64 + lane) * W + w];
            } else {
#pragma unroll
                for (int w = 0; w < W; ++w) a8[w] = an[w];
                if (ks + 1 < ks1) load_operand(ks + 1);
            }
            // -sgn(x_j): a set sign bit (x >= 0) gives -1
            if constexpr (JP != kJFp8) {
                // 16-bit operands: +-1 is 0x3F80 | sign in BF16, 0x3C00 | sign in FP16
                constexpr uint32_t kOne = JP == kJFp16 ? 0x3C003C00u : 0x3F803F80u;
                uint32_t yq[4];  // columns 2q, 2q+1 at bits 0 and 16
#pragma unroll
                for (int q = 0; q < 4; ++q) yq[q] = s8[2 * q] | (s8[2 * q + 1] << 16);
                u32x4 aop[W / 2];  // the terms, largest first
#pragma unroll
                for (int k = 0; k < W / 2; ++k)
                    aop[k] = u32x4{static_cast<uint32_t>(a8[2 * k]), static_cast<uint32_t>(a8[2 * k] >> 32),
                                   static_cast<uint32_t>(a8[2 * k + 1]), static_cast<uint32_t>(a8[2 * k + 1] >> 32)};
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    u32x4 bv;
#pragma unroll
                    for (int q = 0; q < 4; ++q) bv[q] = ((yq[q] << (15 - t)) & 0x80008000u) | kOne;
#pragma unroll
                    for (int k = 0; k < W / 2; ++k) {
                        if constexpr (JP == kJFp16)
                            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                                __builtin_bit_cast(f16x8, bv), __builtin_bit_cast(f16x8, aop[k]), acc[t], 0, 0, 0);
                        else
                            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                __builtin_bit_cast(bf16x8, bv), __builtin_bit_cast(bf16x8, aop[k]), acc[t], 0, 0, 0);
                    }
                }
            } else {
                // byte e of xl / xh: the sign byte of column e / e + 4
                const uint32_t xl = s8[0] | (s8[1] << 8) | (s8[2] << 16) | (s8[3] << 24);
                const uint32_t xh = s8[4] | (s8[5] << 8) | (s8[6] << 16) | (s8[7] << 24);
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    const uint32_t lo = ((xl << (7 - t)) & 0x80808080u) | 0x38383838u;  // e4m3 +-1
                    const uint32_t hi = ((xh << (7 - t)) & 0x80808080u) | 0x38383838u;
                    const long bop = static_cast<long>((static_cast<uint64_t>(hi) << 32) | lo);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(bop, static_cast<long>(a8[0]),
                                                                        acc[t], 0, 0, 0);
                }
            }
        }
    }

    // acc[t][r] = -(sum over the block's columns) for row 16 b + c, agent
    // 128 ab + 16 t + 4 g + r (agents past M are padding: updated, never
    // read back, their sign bits 0)
    const int i = b * kBR + c;
    if (!active || i >= A.n) return;
    const float c0 = static_cast<float>(A.scal[0]);
    const float gk = A.sched[k];
    const float hv = h[i];
    const float sc = JP == kJFp8 ? rowscale[i] : 1.0f;
    uint32_t word = 0;             // byte r, bit t: agent 16 t + 4 g + r
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int m = kMfmaGroup * ab + 16 * t + 4 * g;
        f32x4 xv = xp[t], yv = yp[t];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float xr = xv[r], yr = yv[r];
            sb_update(xr, yr, __builtin_fmaf(-sc, acc[t][r], hv), c0, gk, A.dt, A.dta0);
            xv[r] = xr;
            yv[r] = yr;
            if (m + r < M && xr >= 0.0f) word |= 1u << (8 * r + t);
        }
        st_stream<NT>(xv, reinterpret_cast<f32x4 *>(x + tile + 256 * t));
        st_stream<NT>(yv, reinterpret_cast<f32x4 *>(y + tile + 256 * t));
    }
    reinterpret_cast<uint32_t *>(Sout)[(static_cast<size_t>(i) * R + ab) * 4 + g] = word;
}

size_t mfma_ksteps_bound(int n, int64_t nnz) {
    const size_t nb = (static_cast<size_t>(n) + kBR - 1) / kBR;
    return static_cast<size_t>(nnz) / kBK + nb + 1;
}

hipError_t launch_mfma_plan(int jprec, const StreamArgs &A, const MfmaArgs &P, hipStream_t st) {
    const int nb = (A.n + kBR - 1) / kBR;
    const unsigned gr = static_cast<unsigned>((nb + 255) / 256);
    mfma_count<<<gr, 256, 0, st>>>(A.n, nb, A.row_ptr, A.col, P.kcnt);
    mfma_scan<<<1, kScanThreads, 0, st>>>(nb, P.kcnt, P.koff);
    switch (jprec) {
        case kJFp8: mfma_fill<kJFp8><<<gr, 256, 0, st>>>(nb, A, P.koff, P.kcol, P.kA); break;
        case kJBf16x2: mfma_fill<kJBf16x2><<<gr, 256, 0, st>>>(nb, A, P.koff, P.kcol, P.kA); break;
        case kJFp32: mfma_fill<kJFp32><<<gr, 256, 0, st>>>(nb, A, P.koff, P.kcol, P.kA); break;
        case kJFp8Blk: mfma_fill<kJFp8Blk><<<gr, 256, 0, st>>>(nb, A, P.koff, P.kcol, P.kA); break;
        case kJBf16: mfma_fill<kJBf16><<<gr, 256, 0, st>>>(nb, A, P.koff, P.kcol, P.kA); break;
        case kJFp16: mfma_fill<kJFp16><<<gr, 256, 0, st>>>(nb, A, P.koff, P.kcol, P.kA); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_mfma_state(int n, int M, bool to_tiles, const float *src, float *dst, hipStream_t st) {
    const int64_t runs = static_cast<int64_t>(mfma_state_floats(n, M) / 4);
    if (runs > 0)
        mfma_state<<<static_cast<unsigned>((runs + 255) / 256), 256, 0, st>>>(n, M, to_tiles, src, dst);
    return hipGetLastError();
}

hipError_t launch_mfma_signs(int n, int M, const float *x, uint8_t *S, hipStream_t st) {
    const int64_t total = static_cast<int64_t>(n) * mfma_groups(M) * 16;
    if (total > 0) mfma_signs<<<static_cast<unsigned>((total + 255) / 256), 256, 0, st>>>(n, M, x, S);
    return hipGetLastError();
}

namespace {

template <int JP>
hipError_t launch_mfma_form(const StreamArgs &A, const MfmaArgs &P, int k, float *x, float *y,
                            const uint8_t *Sin, uint8_t *Sout, hipStream_t st) {
    const int nb = (A.n + kBR - 1) / kBR;
    // x and y, FP32, past the caches when larger than the Infinity Cache
    const bool nt = static_cast<size_t>(A.n) * A.M * sizeof(float) * 2 > (size_t(256) << 20);
    const int total = mfma_words(JP) > 1 && nt ? nb * ((mfma_groups(A.M) + 3) / 4)   // shared operands
                                               : (nb + 3) / 4 * mfma_groups(A.M);
    const dim3 grid((total + 7) / 8 * 8);
    if (nt)
        sb_stream_mfma<JP, true><<<grid, 256, 0, st>>>(A, k, P.koff, P.kcol, P.kA, A.h, A.rowscale, x, y,
                                                       Sin, Sout);
    else
        sb_stream_mfma<JP, false><<<grid, 256, 0, st>>>(A, k, P.koff, P.kcol, P.kA, A.h, A.rowscale, x, y,
                                                        Sin, Sout);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_stream_mfma(int jprec, const StreamArgs &A, const MfmaArgs &P, int k, float *x, float *y,
                              const uint8_t *Sin, uint8_t *Sout, hipStream_t st) {
    switch (jprec) {
        case kJFp8: return launch_mfma_form<kJFp8>(A, P, k, x, y, Sin, Sout, st);
        case kJBf16x2: return launch_mfma_form<kJBf16x2>(A, P, k, x, y, Sin, Sout, st);
        case kJFp32: return launch_mfma_form<kJFp32>(A, P, k, x, y, Sin, Sout, st);
        case kJFp8Blk: return launch_mfma_form<kJFp8Blk>(A, P, k, x, y, Sin, Sout, st);
        case kJBf16: return launch_mfma_form<kJBf16>(A, P, k, x, y, Sin, Sout, st);
        case kJFp16: return launch_mfma_form<kJFp16>(A, P, k, x, y, Sin, Sout, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace sbt
