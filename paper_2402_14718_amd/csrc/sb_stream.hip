// Streaming SB step for states that do not fit on chip (gfx950).
//
// Paper section "Simulated Bifurcation": one symplectic-Euler step of bSB
// (Eq. 5-8) or dSB (Eq. 9-12) per launch, all spins and agents at once.
// State x, y is FP32 in HBM, spin-major with agents contiguous.  One wave
// handles one row i for 64 * APL agents (lane l: agents base + 64 k + l), so
// a row's columns and couplings are wave-uniform scalar loads shared by
// all its agents, and every x_j gather is APL coalesced 256-byte lines.
// Rows are padded to multiples of eight couplings (own column, zero
// coupling); each chunk of eight is one scalar load of columns and one of
// couplings, summed in CSR order (the padding adds exact zeros).
//
// dSB reads only the neighbours' signs, kept as 64-bit words -- ballots of
// x >= 0 over 64 agents -- in two alternating planes, so x and y update in
// place and the coupling sum needs no gather of x at all: a sign word is
// itself the lane mask that picks +J_ij or -J_ij for every lane at once.
//
// Workgroups are numbered so that each XCD (workgroups are dealt to the 8
// XCDs round robin) sweeps one contiguous range of rows: neighbouring rows
// share gathered lines, which then stay in that XCD's L2.
//
// Couplings are FP32; FP8 (OCP e4m3) with one FP32 scale per row,
// J_ij = scale_i * e4m3(code_ij), or per block of eight consecutive stored
// couplings of a row (the padded chunk, so one scale per chunk load); or a
// BF16 hi + lo pair per coupling, J_ij = hi + lo (the reduced-precision
// forms).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sb_device.hpp"
#include "sb_kernels.hpp"
#include "sb_stream_kernels.hpp"
#include "sb_stream_chunk.hpp"

namespace sbt {

namespace {

constexpr int kRowsPerWG = 4;  // one row per wave, 256 threads
// Own-row x, y are touched once per step.  When the state is larger than
// the 256 MB Infinity Cache they are streamed past the caches (non-temporal)
// so the gathered x_j lines of neighbouring rows stay in L2; smaller states
// stay cached from one step to the next.
constexpr size_t kStreamNTBytes = size_t(256) << 20;
// bSB with M % 4 == 0: four consecutive agents per lane (16-byte gathers).
constexpr bool kStreamVec4 = true;

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kChunk = kStreamChunk;
constexpr int kPackThreads = 1024;

// Workgroup id -> (row block, agent block), XCD-contiguous.
__device__ __forceinline__ bool map_block(int nrb, int nab, int &rb, int &ab) {
    const int total = nrb * nab;
    const int per_xcd = (total + 7) / 8;
    const int wg = blockIdx.x;
    const int v = (wg % 8) * per_xcd + wg / 8;
    if (v >= total) return false;
    ab = v / nrb;
    rb = v % nrb;
    return true;
}

}  // namespace

// Sign planes from the current positions: S[i * SW + w] bit l =
// x[i, 64 w + l] >= 0 (0 for agents >= M).
__global__ __launch_bounds__(256) void sign_planes(int n, int M, int SW, const float *__restrict__ x,
                                                   uint64_t *__restrict__ S) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * 4 + wave;  // (row, word)
    if (idx >= static_cast<int64_t>(n) * SW) return;
    const int i = static_cast<int>(idx / SW), w = static_cast<int>(idx % SW);
    const int m = w * 64 + lane;
    const bool pos = m < M && x[static_cast<size_t>(i) * M + m] >= 0.0f;
    const uint64_t bal = __ballot(pos);
    if (lane == 0) S[idx] = bal;
}

// Padded row lengths -> row pointers: one workgroup, each thread a
// contiguous range of rows, then a scan over the threads' totals in LDS.
__global__ __launch_bounds__(kPackThreads) void stream_pack_scan(int n, const int *__restrict__ row_ptr,
                                                                  int *__restrict__ prow) {
    __shared__ int tot[kPackThreads];
    const int t = threadIdx.x;
    const int per = (n + kPackThreads - 1) / kPackThreads;
    const int r0 = min(n, t * per), r1 = min(n, r0 + per);
    int sum = 0;
    for (int i = r0; i < r1; ++i) sum += (row_ptr[i + 1] - row_ptr[i] + kChunk - 1) / kChunk * kChunk;
    tot[t] = sum;
    __syncthreads();
    for (int d = 1; d < kPackThreads; d <<= 1) {  // inclusive Hillis-Steele scan
        const int v = t >= d ? tot[t - d] : 0;
        __syncthreads();
        tot[t] += v;
        __syncthreads();
    }
    int at = tot[t] - sum;
    for (int i = r0; i < r1; ++i) {
        prow[i] = at;
        at += (row_ptr[i + 1] - row_ptr[i] + kChunk - 1) / kChunk * kChunk;
    }
    if (t == kPackThreads - 1) prow[n] = tot[t];
}

__global__ __launch_bounds__(256) void stream_pack_fill(int n, const int *__restrict__ row_ptr,
                                                        const int *__restrict__ col,
                                                        const float *__restrict__ J,
                                                        const int *__restrict__ prow,
                                                        int *__restrict__ pcol, float *__restrict__ pJ) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    int q = prow[i];
    for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p, ++q) {
        pcol[q] = col[p];
        pJ[q] = J[p];
    }
    for (; q < prow[i + 1]; ++q) {
        pcol[q] = i;
        pJ[q] = 0.0f;
    }
}

// Per-row FP8 quantisation: scale_i = max_j |J_ij| / 448, code = e4m3(J / scale).
__global__ __launch_bounds__(256) void quantize_fp8_rows(int n, const int *__restrict__ row_ptr,
                                                         const float *__restrict__ J,
                                                         uint8_t *__restrict__ J8,
                                                         float *__restrict__ scale) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float mx = 0.0f;
    for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) mx = fmaxf(mx, __builtin_fabsf(J[p]));
    const float s = mx > 0.0f ? mx / 448.0f : 1.0f;
    scale[i] = s;
    for (int p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
        // |J / s| can round a hair above 448; e4m3's largest finite is 448
        const float q = fminf(fmaxf(J[p] / s, -448.0f), 448.0f);
        J8[p] = static_cast<uint8_t>(__builtin_amdgcn_cvt_pk_fp8_f32(q, q, 0, false) & 0xFF);
    }
}

// FP8 with one FP32 scale per block of kChunk padded couplings:
// scale_b = max |J| over the block / 448 (1 for an all-zero block),
// code = e4m3(J / scale_b) as for the per-row form.
__global__ __launch_bounds__(256) void quantize_fp8_blocks(int64_t nblk, const int *__restrict__ prow_end,
                                                           const float *__restrict__ J,
                                                           uint8_t *__restrict__ J8,
                                                           float *__restrict__ blkscale) {
    const int64_t b = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (b >= nblk || b * kChunk >= *prow_end) return;  // blocks of the padded rows only
    float mx = 0.0f;
    for (int u = 0; u < kChunk; ++u) mx = fmaxf(mx, __builtin_fabsf(J[b * kChunk + u]));
    const float s = mx > 0.0f ? mx / 448.0f : 1.0f;
    blkscale[b] = s;
    for (int u = 0; u < kChunk; ++u) {
        const float q = fminf(fmaxf(J[b * kChunk + u] / s, -448.0f), 448.0f);
        J8[b * kChunk + u] = static_cast<uint8_t>(__builtin_amdgcn_cvt_pk_fp8_f32(q, q, 0, false) & 0xFF);
    }
}

// BF16 to nearest, ties to even, of an FP32 value (its upper 16 bits).
__device__ __forceinline__ uint32_t bf16_bits(float v) {
    const uint32_t u = __float_as_uint(v);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// hi = bf16(J), lo = bf16(J - hi) (the difference is exact in FP32).
__global__ __launch_bounds__(256) void split_bf16x2(int64_t pnnz, const int *__restrict__ prow_end,
                                                    const float *__restrict__ J,
                                                    uint32_t *__restrict__ J2) {
    const int64_t q = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (q >= pnnz || q >= *prow_end) return;  // entries of the padded rows only
    const float j = J[q];
    const uint32_t hi = bf16_bits(j);
    const uint32_t lo = bf16_bits(j - __uint_as_float(hi << 16));
    J2[q] = hi << 16 | lo;
}

template <int MODE, int JP, int APL, bool NT>
__global__ __launch_bounds__(256) void sb_stream(StreamArgs A, int k, const float *xin, float *xout,
                                                 const uint64_t *__restrict__ Sin,
                                                 uint64_t *__restrict__ Sout) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int M = A.M, SW = A.sign_stride;
    const int nrb = (A.n + kRowsPerWG - 1) / kRowsPerWG;
    const int nab = (M + 64 * APL - 1) / (64 * APL);
    int rb, ab;
    if (!map_block(nrb, nab, rb, ab)) return;
    const int i = __builtin_amdgcn_readfirstlane(rb * kRowsPerWG + wave);
    if (i >= A.n) return;
    const int base = ab * 64 * APL;
    bool live[APL];
    int mcol[APL];  // agent column; dead lanes read column 0 (in bounds, one line)
#pragma unroll
    for (int a = 0; a < APL; ++a) {
        const int m = base + 64 * a + lane;
        live[a] = m < M;
        mcol[a] = live[a] ? m : 0;
    }
    const float c0 = static_cast<float>(A.scal[0]);
    const float g = A.sched[k];
    const float scale = JP == kJFp8 ? A.rowscale[i] : 1.0f;
    const int p0 = A.row_ptr[i], p1 = A.row_ptr[i + 1];
    float acc[APL];
#pragma unroll
    for (int a = 0; a < APL; ++a) acc[a] = A.h[i];
    for (int p = p0; p < p1; p += kChunk) {
        const int4 ca = *reinterpret_cast<const int4 *>(A.col + p);
        const int4 cb = *reinterpret_cast<const int4 *>(A.col + p + 4);
        const int c[kChunk] = {ca.x, ca.y, ca.z, ca.w, cb.x, cb.y, cb.z, cb.w};
        float w[kChunk];
        load_chunk<JP>(A, p, scale, w);
        if constexpr (MODE == kDSB) {
#pragma unroll
            for (int u = 0; u < kChunk; ++u) {
                const uint64_t *rec = Sin + static_cast<size_t>(c[u]) * SW + ab * APL;
#pragma unroll
                for (int a = 0; a < APL; ++a) {
                    // J sgn(x_j) = +-J exactly: same value as fma(J, +-1, acc)
                    const bool pos = __builtin_amdgcn_inverse_ballot_w64(rec[a]);
                    acc[a] += pos ? w[u] : -w[u];
                }
            }
        } else {
            float v[kChunk][APL];
#pragma unroll
            for (int u = 0; u < kChunk; ++u) {
                const float *row = xin + static_cast<size_t>(c[u]) * M;
#pragma unroll
                for (int a = 0; a < APL; ++a) v[u][a] = row[mcol[a]];
            }
#pragma unroll
            for (int u = 0; u < kChunk; ++u)
#pragma unroll
                for (int a = 0; a < APL; ++a) acc[a] = __builtin_fmaf(w[u], v[u][a], acc[a]);
        }
    }
    const size_t o = static_cast<size_t>(i) * M;
#pragma unroll
    for (int a = 0; a < APL; ++a) {
        float x = live[a] ? ld_stream<NT>(xin + o + mcol[a]) : 0.0f;
        float y = live[a] ? ld_stream<NT>(A.y + o + mcol[a]) : 0.0f;
        if constexpr (MODE == kASB)
            sb_update_asb(x, y, acc[a], c0, g, A.dt, A.dta0);
        else
            sb_update(x, y, acc[a], c0, g, A.dt, A.dta0);
        if (live[a]) {
            st_stream<NT>(x, xout + o + mcol[a]);
            st_stream<NT>(y, A.y + o + mcol[a]);
        }
        if constexpr (MODE == kDSB) {
            const uint64_t bal = __ballot(live[a] && x >= 0.0f);
            if (lane == 0) Sout[static_cast<size_t>(i) * SW + ab * APL + a] = bal;
        }
    }
}

// bSB / aSB with four consecutive agents per lane (M a multiple of 4): one
// 16-byte gather per coupling and lane, 256 agents per wave.
template <int MODE, int JP, bool NT>
__global__ __launch_bounds__(256) void sb_stream_v4(StreamArgs A, int k, const float *xin,
                                                    float *xout) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int M = A.M;
    const int nrb = (A.n + kRowsPerWG - 1) / kRowsPerWG;
    const int nab = (M + 255) / 256;
    int rb, ab;
    if (!map_block(nrb, nab, rb, ab)) return;
    const int i = __builtin_amdgcn_readfirstlane(rb * kRowsPerWG + wave);
    if (i >= A.n) return;
    const int m = ab * 256 + 4 * lane;
    const bool live = m < M;
    const int mcol = live ? m : 0;  // dead lanes read agents 0..3 (in bounds)
    const float c0 = static_cast<float>(A.scal[0]);
    const float g = A.sched[k];
    const float scale = JP == kJFp8 ? A.rowscale[i] : 1.0f;
    const int p0 = A.row_ptr[i], p1 = A.row_ptr[i + 1];
    float4 acc = make_float4(A.h[i], A.h[i], A.h[i], A.h[i]);
    for (int p = p0; p < p1; p += kChunk) {
        const int4 ca = *reinterpret_cast<const int4 *>(A.col + p);
        const int4 cb = *reinterpret_cast<const int4 *>(A.col + p + 4);
        const int c[kChunk] = {ca.x, ca.y, ca.z, ca.w, cb.x, cb.y, cb.z, cb.w};
        float w[kChunk];
        load_chunk<JP>(A, p, scale, w);
        float4 v[kChunk];
#pragma unroll
        for (int u = 0; u < kChunk; ++u)
            v[u] = *reinterpret_cast<const float4 *>(xin + static_cast<size_t>(c[u]) * M + mcol);
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            acc.x = __builtin_fmaf(w[u], v[u].x, acc.x);
            acc.y = __builtin_fmaf(w[u], v[u].y, acc.y);
            acc.z = __builtin_fmaf(w[u], v[u].z, acc.z);
            acc.w = __builtin_fmaf(w[u], v[u].w, acc.w);
        }
    }
    if (!live) return;
    const size_t o = static_cast<size_t>(i) * M + mcol;
    const f32x4 xv = ld_stream<NT>(reinterpret_cast<const f32x4 *>(xin + o));
    const f32x4 yv = ld_stream<NT>(reinterpret_cast<const f32x4 *>(A.y + o));
    float x[4] = {xv.x, xv.y, xv.z, xv.w}, y[4] = {yv.x, yv.y, yv.z, yv.w};
    const float f[4] = {acc.x, acc.y, acc.z, acc.w};
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        if constexpr (MODE == kASB)
            sb_update_asb(x[a], y[a], f[a], c0, g, A.dt, A.dta0);
        else
            sb_update(x[a], y[a], f[a], c0, g, A.dt, A.dta0);
    }
    st_stream<NT>(f32x4{x[0], x[1], x[2], x[3]}, reinterpret_cast<f32x4 *>(xout + o));
    st_stream<NT>(f32x4{y[0], y[1], y[2], y[3]}, reinterpret_cast<f32x4 *>(A.y + o));
}

hipError_t launch_sign_planes(int n, int M, const float *x, uint64_t *S, hipStream_t st) {
    const int SW = stream_sign_stride(M);
    const int64_t words = static_cast<int64_t>(n) * SW;
    sign_planes<<<static_cast<unsigned>((words + 3) / 4), 256, 0, st>>>(n, M, SW, x, S);
    return hipGetLastError();
}

hipError_t launch_stream_pack(int n, const int *row_ptr, const int *col, const float *J, int *prow,
                              int *pcol, float *pJ, hipStream_t st) {
    stream_pack_scan<<<1, kPackThreads, 0, st>>>(n, row_ptr, prow);
    stream_pack_fill<<<(n + 255) / 256, 256, 0, st>>>(n, row_ptr, col, J, prow, pcol, pJ);
    return hipGetLastError();
}

hipError_t launch_quantize_fp8_blocks(int n, const int *prow, int64_t pnnz, const float *J,
                                      uint8_t *J8, float *blkscale, hipStream_t st) {
    const int64_t nblk = pnnz / kChunk;
    if (nblk > 0)
        quantize_fp8_blocks<<<static_cast<unsigned>((nblk + 255) / 256), 256, 0, st>>>(
            nblk, prow + n, J, J8, blkscale);
    return hipGetLastError();
}

hipError_t launch_split_bf16x2(int n, const int *prow, int64_t pnnz, const float *J, uint32_t *J2,
                               hipStream_t st) {
    if (pnnz > 0)
        split_bf16x2<<<static_cast<unsigned>((pnnz + 255) / 256), 256, 0, st>>>(pnnz, prow + n, J,
                                                                              J2);
    return hipGetLastError();
}

hipError_t launch_quantize_fp8(int n, const int *row_ptr, const float *J, uint8_t *J8, float *scale,
                               hipStream_t st) {
    quantize_fp8_rows<<<(n + 255) / 256, 256, 0, st>>>(n, row_ptr, J, J8, scale);
    return hipGetLastError();
}

namespace {

template <int MODE, int JP, bool NT>
hipError_t launch_stream_apl(const StreamArgs &A, int k, const float *xin, float *xout,
                             const uint64_t *Sin, uint64_t *Sout, hipStream_t st) {
    const int apl = stream_apl(A.M, MODE);
    const int nrb = (A.n + kRowsPerWG - 1) / kRowsPerWG;
    const int total = nrb * ((A.M + 64 * apl - 1) / (64 * apl));
    const int grid = (total + 7) / 8 * 8;
    switch (apl) {
        case 8: sb_stream<MODE, JP, 8, NT><<<grid, 256, 0, st>>>(A, k, xin, xout, Sin, Sout); break;
        case 4: sb_stream<MODE, JP, 4, NT><<<grid, 256, 0, st>>>(A, k, xin, xout, Sin, Sout); break;
        case 2: sb_stream<MODE, JP, 2, NT><<<grid, 256, 0, st>>>(A, k, xin, xout, Sin, Sout); break;
        default: sb_stream<MODE, JP, 1, NT><<<grid, 256, 0, st>>>(A, k, xin, xout, Sin, Sout); break;
    }
    return hipGetLastError();
}

// bSB / aSB: neighbours' positions gathered
template <int MODE, bool NT>
hipError_t launch_stream_gather(int jprec, const StreamArgs &A, int k, const float *xin, float *xout,
                                hipStream_t st) {
    if (kStreamVec4 && A.M % 4 == 0 && A.M > 64) {
        const int nrb = (A.n + kRowsPerWG - 1) / kRowsPerWG;
        const int total = nrb * ((A.M + 255) / 256);
        const int grid = (total + 7) / 8 * 8;
        if (jprec == kJFp8)
            sb_stream_v4<MODE, kJFp8, NT><<<grid, 256, 0, st>>>(A, k, xin, xout);
        else if (jprec == kJFp8Blk)
            sb_stream_v4<MODE, kJFp8Blk, NT><<<grid, 256, 0, st>>>(A, k, xin, xout);
        else if (jprec == kJBf16x2)
            sb_stream_v4<MODE, kJBf16x2, NT><<<grid, 256, 0, st>>>(A, k, xin, xout);
        else
            sb_stream_v4<MODE, kJFp32, NT><<<grid, 256, 0, st>>>(A, k, xin, xout);
        return hipGetLastError();
    }
    switch (jprec) {
        case kJFp8: return launch_stream_apl<MODE, kJFp8, NT>(A, k, xin, xout, nullptr, nullptr, st);
        case kJFp8Blk: return launch_stream_apl<MODE, kJFp8Blk, NT>(A, k, xin, xout, nullptr, nullptr, st);
        case kJBf16x2: return launch_stream_apl<MODE, kJBf16x2, NT>(A, k, xin, xout, nullptr, nullptr, st);
        default: return launch_stream_apl<MODE, kJFp32, NT>(A, k, xin, xout, nullptr, nullptr, st);
    }
}

template <bool NT>
hipError_t launch_stream_nt(int mode, int jprec, const StreamArgs &A, int k, const float *xin,
                            float *xout, const uint64_t *Sin, uint64_t *Sout, hipStream_t st) {
    if (mode == kDSB) switch (jprec) {
            case kJFp8: return launch_stream_apl<kDSB, kJFp8, NT>(A, k, xin, xout, Sin, Sout, st);
            case kJFp8Blk: return launch_stream_apl<kDSB, kJFp8Blk, NT>(A, k, xin, xout, Sin, Sout, st);
            case kJBf16x2: return launch_stream_apl<kDSB, kJBf16x2, NT>(A, k, xin, xout, Sin, Sout, st);
            default: return launch_stream_apl<kDSB, kJFp32, NT>(A, k, xin, xout, Sin, Sout, st);
        }
    return mode == kASB ? launch_stream_gather<kASB, NT>(jprec, A, k, xin, xout, st)
                        : launch_stream_gather<kBSB, NT>(jprec, A, k, xin, xout, st);
}

}  // namespace

hipError_t launch_stream2(int mode, int jprec, const StreamArgs &A, int k, const float *xin,
                          float *xout, const uint64_t *Sin, uint64_t *Sout, hipStream_t st) {
    // x (once or twice) and y, FP32
    const size_t state = static_cast<size_t>(A.n) * A.M * sizeof(float) * (mode == kDSB ? 2 : 3);
    return state > kStreamNTBytes ? launch_stream_nt<true>(mode, jprec, A, k, xin, xout, Sin, Sout, st)
                                  : launch_stream_nt<false>(mode, jprec, A, k, xin, xout, Sin, Sout, st);
}

}  // namespace sbt
