// Coupling chunks of the streaming steps (sb_stream.hip, sb_stream_tile.hip):
// the padded CSR rows are read eight couplings at a time, each chunk one
// aligned load, decoded to FP32 from the stored form.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "sb_kernels.hpp"
#include "sb_stream_kernels.hpp"

namespace sbt {

// FP8 e4m3 (OCP) byte `sel` of a dword -> FP32 on the conversion unit.
template <int SEL>
__device__ __forceinline__ float e4m3_to_f32(uint32_t word) {
    return __builtin_amdgcn_cvt_f32_fp8(static_cast<int>(word), SEL);
}

// The BF16 pair of a coupling as FP32: hi + lo (exact in FP32: lo is the
// rounded remainder of hi, at most 16 significant bits below it).
__device__ __forceinline__ float bf16x2_value(uint32_t w) {
    return __uint_as_float(w & 0xFFFF0000u) + __uint_as_float(w << 16);
}

// Couplings p .. p + kStreamChunk - 1 (p a multiple of kStreamChunk) as
// FP32; `scale` is the row's FP8 scale (per-row form only).
template <int JP>
__device__ __forceinline__ void load_chunk(const StreamArgs &A, int p, float scale,
                                           float (&w)[kStreamChunk]) {
    static_assert(kStreamChunk == 8, "chunks are two dwords of FP8 codes");
    if constexpr (JP == kJFp8 || JP == kJFp8Blk) {
        if constexpr (JP == kJFp8Blk) scale = A.blkscale[p / kStreamChunk];
        const uint2 codes = *reinterpret_cast<const uint2 *>(A.J8 + p);
        w[0] = scale * e4m3_to_f32<0>(codes.x);
        w[1] = scale * e4m3_to_f32<1>(codes.x);
        w[2] = scale * e4m3_to_f32<2>(codes.x);
        w[3] = scale * e4m3_to_f32<3>(codes.x);
        w[4] = scale * e4m3_to_f32<0>(codes.y);
        w[5] = scale * e4m3_to_f32<1>(codes.y);
        w[6] = scale * e4m3_to_f32<2>(codes.y);
        w[7] = scale * e4m3_to_f32<3>(codes.y);
    } else if constexpr (JP == kJBf16x2) {
        const uint4 a = *reinterpret_cast<const uint4 *>(A.J2 + p);
        const uint4 b = *reinterpret_cast<const uint4 *>(A.J2 + p + 4);
        const uint32_t v[kStreamChunk] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (int u = 0; u < kStreamChunk; ++u) w[u] = bf16x2_value(v[u]);
    } else {
#pragma unroll
        for (int u = 0; u < kStreamChunk; ++u) w[u] = A.J[p + u];
    }
}

// Own-row x, y: streamed past the caches (non-temporal) when the state is
// larger than the Infinity Cache, plain loads and stores otherwise.
template <bool NT, class T>
__device__ __forceinline__ T ld_stream(const T *p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <bool NT, class T>
__device__ __forceinline__ void st_stream(T v, T *p) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

}  // namespace sbt
