// Matrix-core dSB streaming step (sb_stream_mfma.hip): argument block,
// plan and step launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "sb_kernels.hpp"
#include "sb_stream_kernels.hpp"

namespace sbt {

// A block is kMfmaRows consecutive rows: the M side of one 16 x 16 output
// tile of the matrix instruction.  Its distinct columns are listed in
// ascending order and padded to whole K-steps of kMfmaK columns (the
// instruction's contraction length); each K-step holds the block's
// couplings on those columns as one dense operand tile, already in the
// instruction's register layout (lane 16 g + r holds row r's couplings on
// listed columns 8 g .. 8 g + 7 of the step; 0 where the row has none).
// FP32 couplings are split exactly into three BF16 terms, J = hi + mid + lo
// (8 significant bits each), three operands on the same signs; FP8 with a
// scale per block of 8 couplings is decoded to the FP32 value the CSR step
// uses (scale x code) and split the same way.  BF16 and FP16 couplings
// (the batch functions' forms) are one operand each.
constexpr int kMfmaRows = 16;
constexpr int kMfmaK = 32;

// 64-bit words of one lane's operand per K-step: eight FP8 codes (one
// word), eight BF16 hi then eight BF16 lo (four words), or eight BF16 hi,
// mid and lo of FP32 (or block-scaled FP8) couplings (six words).
__host__ __device__ constexpr int mfma_words(int jprec) {
    return jprec == kJBf16x2 ? 4
           : (jprec == kJFp32 || jprec == kJFp8Blk) ? 6
           : (jprec == kJBf16 || jprec == kJFp16) ? 2
                                                   : 1;
}

// Coupling forms the matrix-core step takes: FP8 with one scale per row
// (the codes are the operand, the scale applies to the row's sum), the
// BF16 hi + lo pair, FP32 and FP8 with a scale per block of 8 (two or three
// BF16 operands on the same signs), BF16 and FP16 (one operand).
__host__ __device__ constexpr bool mfma_form(int jprec) {
    return jprec == kJFp8 || jprec == kJBf16x2 || jprec == kJFp32 || jprec == kJFp8Blk ||
           jprec == kJBf16 || jprec == kJFp16;
}

struct MfmaArgs {
    int *kcnt;       // [nb] K-steps of each block (work array of the plan)
    int *koff;       // [nb + 1] first K-step of each block; koff[nb] = total
    int *kcol;       // [ksteps * kMfmaK] listed columns
    uint64_t *kA;    // [ksteps * 64 * mfma_words] operand tiles
};

// Sign records of the matrix-core step (its own layout, not the CSR step's
// sign words): per row and group of kMfmaGroup agents 16 bytes, bit t of
// byte c = (x of agent kMfmaGroup g + 16 t + c >= 0), 0 past the last agent.
// A lane of the step handles agent c of each of the group's 8 tiles of 16,
// so one byte holds all its signs of one column, and the new signs of its
// row are one byte it writes itself.
constexpr int kMfmaGroup = 128;
__host__ __device__ constexpr int mfma_groups(int M) { return (M + kMfmaGroup - 1) / kMfmaGroup; }
__host__ __device__ constexpr size_t mfma_sign_bytes(int n, int M) {
    return static_cast<size_t>(n) * mfma_groups(M) * 16;
}
hipError_t launch_mfma_signs(int n, int M, const float *x, uint8_t *S, hipStream_t st);

// The step's own layout of x and y: each (block of kMfmaRows rows, group of
// kMfmaGroup agents) is one contiguous tile of 2048 floats, in the order the
// step's lanes touch them -- element (row 16 b + c, agent 128 a + 16 t + 4 g
// + r) at (b R + a) 2048 + 256 t + 4 (16 g + c) + r, R = mfma_groups(M) --
// so every 16-byte access of a wave falls in one 1 KB run.  Rows are padded
// to whole blocks and agents to whole groups (the padding is zero and never
// read back).  Converted from and to the spin-major layout (x[i M + m]) of
// the other kernels at the start, at energy checkpoints and at the end.
__host__ __device__ constexpr size_t mfma_state_floats(int n, int M) {
    return static_cast<size_t>((n + kMfmaRows - 1) / kMfmaRows) * mfma_groups(M) * kMfmaRows * kMfmaGroup;
}
// to_tiles: spin-major src -> tiled dst (padding zeroed); else tiled src ->
// spin-major dst.
hipError_t launch_mfma_state(int n, int M, bool to_tiles, const float *src, float *dst, hipStream_t st);

// Upper bound on the K-steps of all blocks: a block lists at most its own
// couplings, padded by fewer than kMfmaK.
size_t mfma_ksteps_bound(int n, int64_t nnz);
hipError_t launch_mfma_plan(int jprec, const StreamArgs &A, const MfmaArgs &P, hipStream_t st);
// One dSB step on the tiled x, y (mfma_state_floats each), in place; the
// neighbours' signs are read from the records Sin and the new signs written
// to Sout (mfma_sign_bytes each).
hipError_t launch_stream_mfma(int jprec, const StreamArgs &A, const MfmaArgs &P, int k, float *x, float *y,
                              const uint8_t *Sin, uint8_t *Sout, hipStream_t st);

}  // namespace sbt
