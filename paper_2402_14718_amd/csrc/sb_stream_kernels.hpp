// Argument blocks and launchers of the streaming SB steps (one launch per
// step, state in HBM): the one-row and row-quad steps (sb_stream.hip,
// sb_stream_quad.hip), the tiled step (sb_stream_tile.hip) and their
// one-off preparation of the couplings.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "sb_kernels.hpp"

namespace sbt {

// Streaming kernel's couplings: CSR with every row padded to a multiple of
// kStreamChunk entries by (own column, zero coupling), so each chunk of
// columns and couplings is one aligned scalar load.
constexpr int kStreamChunk = 8;

// Agents per lane of the streaming kernel: one wave covers one row for
// 64 * APL agents, lane l holding agents base + 64 k + l (k < APL), so the
// row's dSB sign words for those agents are APL consecutive 64-bit words.
// Largest APL per form (bSB: gathers in flight vs VGPRs; dSB: sign
// records in flight vs SGPRs).
constexpr int kStreamAplMaxBsb = 4;
constexpr int kStreamAplMaxDsb = 8;
__host__ __device__ constexpr int stream_apl(int M, int mode) {
    const int cap = mode == 1 ? kStreamAplMaxDsb : kStreamAplMaxBsb;  // dSB : bSB, aSB
    const int apl = M > 256 ? 8 : (M > 128 ? 4 : (M > 64 ? 2 : 1));
    return apl < cap ? apl : cap;
}
// 64-bit dSB sign words per spin: ceil(M / 64) rounded up to a multiple of APL.
__host__ __device__ constexpr int stream_sign_stride(int M) {
    return ((M + 63) / 64 + stream_apl(M, 1) - 1) / stream_apl(M, 1) * stream_apl(M, 1);
}

struct StreamArgs {
    int n, M, K;
    double a0;
    float dt, dta0;
    const int *row_ptr;          // [n+1] padded row pointers (multiples of kStreamChunk)
    const int *col;              // [padded nnz]
    const float *J;              // [padded nnz] FP32 couplings
    const float *h;
    const double *scal;
    float *y;
    const float *sched;          // [K] a0 - a_k
    const uint8_t *J8;           // [padded nnz] FP8 e4m3 couplings (FP8 forms)
    const float *rowscale;       // [n] per-row FP32 scale of J8
    const float *blkscale;       // [padded nnz / kStreamChunk] per-block scale of J8
    const uint32_t *J2;          // [padded nnz] BF16 hi << 16 | BF16 lo
    int sign_stride;             // stream_sign_stride(M)
};

// Row quads of the streaming bSB / aSB step (sb_stream_quad.hip): each
// quad of kQuadRows consecutive rows lists its distinct columns ascending
// (padded to whole chunks of kStreamChunk) with one FP32 coupling per row
// and column (0 where the row has none).
constexpr int kQuadRows = 4;

struct QuadArgs {
    int *qcnt;                   // [nq] listed columns per quad (work array of the plan)
    int *qoff;                   // [nq+1] first listed column of each quad
    int *qcol;                   // [quad_cols_bound] listed columns
    float *qJ;                   // [quad_cols_bound * kQuadRows] couplings, column-major
};

size_t quad_cols_bound(int n, int64_t nnz);
hipError_t launch_quad_plan(int jprec, const StreamArgs &A, const QuadArgs &Q, hipStream_t st);
hipError_t launch_stream_quad(int mode, const StreamArgs &A, const QuadArgs &Q, int k, const float *xin,
                              float *xout, hipStream_t st);

// Row tiles of the streaming bSB / aSB step (sb_stream_tile.hip): super
// tiles of kTileSuper consecutive rows, each cut into tiles of consecutive
// rows whose column union has at most `ucap` (<= kTileColsMax) entries and
// whose padded couplings number at most kTileNnz; per step a tile's union
// positions (64 agents x 4 B per column) and its couplings are staged in LDS.
constexpr int kTileSuper = 32;
constexpr int kTileColsMax = 256;
constexpr int kTileColsDefault = 192;
constexpr int kTileNnz = 640;
constexpr uint16_t kTileGlobal = 0xFFFF;  // ploc of a tile read from global memory
__host__ __device__ constexpr size_t tile_lds_bytes(int ucap) {
    return sizeof(float) * 64 * static_cast<size_t>(ucap) + (sizeof(float) + sizeof(uint16_t)) * kTileNnz;
}

struct TileArgs {
    int ucap;                    // columns a tile stages, kStreamChunk .. kTileColsMax
    int2 *tile_info;             // [nsuper * kTileSuper] (first row, union size) per tile
    int *tile_n;                 // [nsuper] tiles of each super tile
    int *tile_cols;              // [padded nnz] a tile's union, ascending, stored from its
                                 //   first row's padded row pointer on
    uint16_t *ploc;              // [padded nnz] index of the coupling's column in its
                                 //   tile's union (kTileGlobal: tile read from global)
};

hipError_t launch_tile_plan(int n, const int *prow, const int *pcol, const TileArgs &T,
                            hipStream_t st);
hipError_t launch_stream_tile(int mode, int jprec, const StreamArgs &A, const TileArgs &T, int k,
                              const float *xin, float *xout, hipStream_t st);

hipError_t launch_stream2(int mode, int jprec, const StreamArgs &A, int k, const float *xin,
                          float *xout, const uint64_t *Sin, uint64_t *Sout, hipStream_t st);
hipError_t launch_sign_planes(int n, int M, const float *x, uint64_t *S, hipStream_t st);
// FP8 with one scale per block of kStreamChunk padded couplings; BF16 hi +
// lo pairs (both over the padded rows)
// (over the padded rows: prow[n] entries of capacity pnnz)
hipError_t launch_quantize_fp8_blocks(int n, const int *prow, int64_t pnnz, const float *J,
                                      uint8_t *J8, float *blkscale, hipStream_t st);
hipError_t launch_split_bf16x2(int n, const int *prow, int64_t pnnz, const float *J, uint32_t *J2,
                               hipStream_t st);
hipError_t launch_quantize_fp8(int n, const int *row_ptr, const float *J, uint8_t *J8, float *scale,
                               hipStream_t st);
// Padded copy (col, J) -> (pcol, pJ) with row pointers prow; pcol and pJ hold
// at most nnz + (kStreamChunk - 1) n entries.
hipError_t launch_stream_pack(int n, const int *row_ptr, const int *col, const float *J, int *prow,
                              int *pcol, float *pJ, hipStream_t st);

}  // namespace sbt
