// Device-side building blocks shared by the SB kernels: the Philox draw of
// the initial state and the fused symplectic-Euler update of one
// (spin, agent) pair.  Both step kernels (resident and streaming) call the
// same update with the same operation order, so they produce bit-identical
// trajectories.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sbt {

enum : int { kBSB = 0, kDSB = 1, kASB = 2 };

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
// (hi0, lo0) = M0 c0, (hi1, lo1) = M1 c2, c = (hi1^c1^k0, lo1, hi0^c3^k1, lo0),
// bumping the key by the Weyl constants between rounds.
struct Philox4 {
    uint32_t v[4];
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t hi0 = static_cast<uint32_t>(p0 >> 32), lo0 = static_cast<uint32_t>(p0);
        const uint32_t hi1 = static_cast<uint32_t>(p1 >> 32), lo1 = static_cast<uint32_t>(p1);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Philox4 o;
    o.v[0] = c0;
    o.v[1] = c1;
    o.v[2] = c2;
    o.v[3] = c3;
    return o;
}

// ((r >> 8) - 2^23) * 2^-26: uniform on [-1/8, 1/8), exact in FP32.
__device__ __forceinline__ float philox_word_to_unit(uint32_t r) {
    return static_cast<float>(static_cast<int32_t>(r >> 8) - (1 << 23)) * 0x1p-26f;
}

// sgn(x) with sgn(0) = +1, as copysign(1, x): one bitfield insert.  The
// two differ only at x = -0, which no position ever holds: starts are +0 or
// nonzero, and the steps' fused multiply-adds and clamp return -0 only
// when their addend already is -0.
__device__ __forceinline__ float sgnf(float v) { return __builtin_copysignf(1.0f, v); }

// Schedule factor (a0 - a_k) with a_k = a0 k / K, evaluated in FP64.
__device__ __forceinline__ float schedule_gap(double a0, int k, int K) {
    return static_cast<float>(a0 - a0 * static_cast<double>(k) / static_cast<double>(K));
}

// One symplectic-Euler step of one oscillator (Eq. 5-6 / 9-10) followed by
// the inelastic wall (Eq. 8 / 12):
//   y += dt (c0 F - g x),  x += dt a0 y,  |x| > 1 -> x = sgn(x), y = 0.
// F holds h_i + sum_j J_ij op(x_j) (the field seeds the sum).  Rounding is
// pinned with explicit fused multiply-adds.  Past the wall, sgn(x) equals
// x clamped to [-1, 1] (one v_med3), and inside it the clamp is exact.
__device__ __forceinline__ void sb_update(float &x, float &y, float F, float c0, float g,
                                          float dt, float dta0) {
    const float gx = g * x;
    const float force = __builtin_fmaf(c0, F, -gx);
    const float yn = __builtin_fmaf(dt, force, y);
    const float xn = __builtin_fmaf(dta0, yn, x);
    const bool wall = __builtin_fabsf(xn) > 1.0f;
    x = __builtin_amdgcn_fmed3f(xn, -1.0f, 1.0f);
    y = wall ? 0.0f : yn;
}

// One symplectic-Euler step of aSB (Eq. 1-2), no wall:
//   y += dt (c0 F - (x^2 + g) x),  x += dt a0 y.
__device__ __forceinline__ void sb_update_asb(float &x, float &y, float F, float c0, float g,
                                              float dt, float dta0) {
    const float q = __builtin_fmaf(x, x, g);
    const float force = __builtin_fmaf(c0, F, -(q * x));
    y = __builtin_fmaf(dt, force, y);
    x = __builtin_fmaf(dta0, y, x);
}

// The step of the mode: aSB (no wall) or bSB / dSB (wall).
template <int MODE>
__device__ __forceinline__ void sb_step(float &x, float &y, float F, float c0, float g, float dt,
                                        float dta0) {
    if constexpr (MODE == kASB)
        sb_update_asb(x, y, F, c0, g, dt, dta0);
    else
        sb_update(x, y, F, c0, g, dt, dta0);
}

// What the coupling reads of a neighbour: its position (bSB, Eq. 6; aSB) or
// its sign (dSB, Eq. 10).
template <int MODE>
__device__ __forceinline__ float shared_value(float x) {
    if constexpr (MODE == kDSB)
        return sgnf(x);
    else
        return x;
}

// ------------------------------------------------------------ reductions

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return __builtin_amdgcn_readfirstlane(v);
}

// Exclusive prefix sum over the workgroup (thread order) of one int per
// thread; `total` receives the sum over all threads.  `wsum` holds one int
// per wave.  The workgroup size must be a multiple of 64, and every thread
// must call it.
__device__ __forceinline__ int block_exclusive_scan(int v, int *wsum, int &total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = static_cast<int>(blockDim.x) >> 6;
    int x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    int base = 0;
    total = 0;
    for (int w = 0; w < nw; ++w) {
        const int s = wsum[w];
        if (w < wave) base += s;
        total += s;
    }
    __syncthreads();
    return base + x - v;
}

// Deterministic sum over the workgroup of one double per thread (fixed
// tree order); the result is valid in thread 0.  `red` holds one double
// per wave.  Every thread of the workgroup must call it.
__device__ __forceinline__ double block_sum(double v, double *red) {
    v = wave_sum(v);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = static_cast<int>(blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; ++w) s += red[w];
    }
    __syncthreads();
    return s;
}

// Records the largest dynamic-LDS size a kernel has been opened up to, so
// the attribute is set once (on a kernel's first launch) rather than on
// every launch -- launches may be captured into a HIP graph.
bool lds_attribute_needed(const void *fn, size_t lds);

// Launch with a dynamic-LDS request beyond the default limit.
template <class F, class... Args>
hipError_t launch_with_lds(F fn, dim3 grid, dim3 block, size_t lds, hipStream_t st, Args... args) {
    if (lds_attribute_needed(reinterpret_cast<const void *>(fn), lds)) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    fn<<<grid, block, lds, st>>>(args...);
    return hipGetLastError();
}

}  // namespace sbt
