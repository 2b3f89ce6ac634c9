// Host orchestration of the SB solver: argument checks, workspace layout,
// kernel selection and the sbt_solve / sbt_solve_dev entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

#include "common.hpp"
#include "sb_kernels.hpp"
#include "sb_stream_kernels.hpp"
#include "sb_stream_mfma.hpp"
#include "sbtrack.h"

namespace {

using sbt::fail;

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t J = 0, h = 0, scal = 0, prep = 0, perm = 0, sched = 0, xa = 0, xb = 0, y = 0, epart = 0,
           etrace = 0, S0 = 0, S1 = 0, J8 = 0, rowscale = 0, prow = 0, pcol = 0, pJ = 0,
           tile_info = 0, tile_n = 0, tile_cols = 0, ploc = 0, blkscale = 0, J2 = 0, qcnt = 0,
           qoff = 0, qcol = 0, qJ = 0, kcnt = 0, koff = 0, kcol = 0, kA = 0, xt = 0, yt = 0;
    size_t total = 0;
    int n_ckpt = 0;
};

// x is updated in place under dSB (the streaming kernel's neighbours are
// the sign planes S0/S1), so the second position buffer exists for bSB
// only; FP8 couplings add one byte per padded nonzero and a scale per row.
// prow/pcol/pJ: the streaming kernel's row-padded copy of the couplings;
// the tiled step (requested explicitly) adds its tile plan, the bSB / aSB
// streaming step over row quads (four agents per lane) its quad lists.
// bSB / aSB streaming (SBT_KERNEL_STREAM) runs over row quads when whole
// lanes of four agents fill more than one wave; otherwise, and on request
// (SBT_KERNEL_STREAM_ROWS), over single rows (sb_stream.hip).  The
// matrix-core dSB step (requested explicitly) adds its block lists and
// operand tiles.
bool quad_step(sbt_mode mode, int32_t M) { return mode != SBT_DSB && M % 4 == 0 && M > 64; }

// AUTO runs dSB on the matrix-core step from 2^23 spin-agent pairs on, for
// every streaming coupling form (measured against the CSR step, FP8 /
// BF16X2 / FP32 / FP8_BLOCK: 208710 x 512, 1.92x / 1.68x / 1.46x / 1.43x;
// 8493 x 1024, cache-resident, 1.33x / 1.06x / 1.09x / 1.24x; 1480 x 256
// is launch-bound and the matrix-core step 0.86x / 0.85x / 0.84x / 0.82x).
// FP16 and BF16 single solves run only there (the CSR steps do not take
// them; the batch functions do).
constexpr size_t kMfmaAutoPairs = size_t(1) << 23;
bool mfma_auto(sbt_mode mode, int32_t prec, int32_t n, int32_t M) {
    return mode == SBT_DSB && static_cast<size_t>(n) * static_cast<size_t>(M) >= kMfmaAutoPairs;
}

Layout make_layout(int32_t n, int64_t nnz, int32_t M, int32_t K, int32_t every, sbt_mode mode,
                   int32_t prec, int32_t kernel_req) {
    const bool tiled = kernel_req == SBT_KERNEL_STREAM_TILE;
    // (AUTO may resolve to the streaming step, so it reserves the lists too)
    const bool quads = quad_step(mode, M) &&
                       (kernel_req == SBT_KERNEL_STREAM || kernel_req == SBT_KERNEL_AUTO);
    const bool mfma = (kernel_req == SBT_KERNEL_STREAM_MFMA && mode == SBT_DSB) ||
                      (kernel_req == SBT_KERNEL_AUTO && mfma_auto(mode, prec, n, M));
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + std::max<size_t>(bytes, 1));
        return at;
    };
    const size_t nm = static_cast<size_t>(n) * static_cast<size_t>(M);
    const size_t nblk_prep = (static_cast<size_t>(n) + 255) / 256;
    const size_t nblk_e = (static_cast<size_t>(n) + sbt::kEnergyRows - 1) / sbt::kEnergyRows;
    L.n_ckpt = every > 0 ? K / every : 0;
    L.J = take(sizeof(float) * static_cast<size_t>(nnz));
    L.h = take(sizeof(float) * n);
    L.scal = take(sizeof(double) * 8);
    L.prep = take(sizeof(double) * 4 * nblk_prep);
    L.perm = take(sizeof(int32_t) * n);
    L.sched = take(sizeof(float) * static_cast<size_t>(K));
    L.xa = take(sizeof(float) * nm);
    L.xb = mode != SBT_DSB ? take(sizeof(float) * nm) : L.xa;
    L.y = take(sizeof(float) * nm);
    L.epart = take(sizeof(double) * nblk_e * M);
    L.etrace = take(sizeof(double) * static_cast<size_t>(L.n_ckpt) * M);
    if (mode == SBT_DSB) {
        // the CSR step's sign words, or the matrix-core step's sign records
        const size_t bytes = mfma ? sbt::mfma_sign_bytes(n, M)
                                  : sizeof(uint64_t) * static_cast<size_t>(n) * sbt::stream_sign_stride(M);
        L.S0 = take(bytes);
        L.S1 = take(bytes);
    }
    const size_t pnnz = static_cast<size_t>(nnz) + (sbt::kStreamChunk - 1) * static_cast<size_t>(n);
    L.prow = take(sizeof(int32_t) * (static_cast<size_t>(n) + 1));
    L.pcol = take(sizeof(int32_t) * pnnz);
    L.pJ = take(sizeof(float) * pnnz);
    if (prec == SBT_PREC_FP8) {
        L.J8 = take(pnnz);
        L.rowscale = take(sizeof(float) * n);
    }
    if (prec == SBT_PREC_FP8_BLOCK) {
        L.J8 = take(pnnz);
        L.blkscale = take(sizeof(float) * (pnnz / sbt::kStreamChunk));
    }
    if (prec == SBT_PREC_BF16X2) L.J2 = take(sizeof(uint32_t) * pnnz);
    if (quads) {  // the row-quad streaming step's lists
        const size_t nq = (static_cast<size_t>(n) + sbt::kQuadRows - 1) / sbt::kQuadRows;
        const size_t cols = sbt::quad_cols_bound(n, nnz);
        L.qcnt = take(sizeof(int32_t) * nq);
        L.qoff = take(sizeof(int32_t) * (nq + 1));
        L.qcol = take(sizeof(int32_t) * cols);
        L.qJ = take(sizeof(float) * cols * sbt::kQuadRows);
    }
    if (mfma) {  // the matrix-core step's blocks and operand tiles
        const size_t nb = (static_cast<size_t>(n) + sbt::kMfmaRows - 1) / sbt::kMfmaRows;
        const size_t ks = sbt::mfma_ksteps_bound(n, nnz);
        const int jp = prec == SBT_PREC_FP8         ? sbt::kJFp8
                       : prec == SBT_PREC_BF16X2    ? sbt::kJBf16x2
                       : prec == SBT_PREC_FP8_BLOCK ? sbt::kJFp8Blk
                       : prec == SBT_PREC_BF16      ? sbt::kJBf16
                       : prec == SBT_PREC_FP16      ? sbt::kJFp16
                                                    : sbt::kJFp32;
        L.kcnt = take(sizeof(int32_t) * nb);
        L.koff = take(sizeof(int32_t) * (nb + 1));
        L.kcol = take(sizeof(int32_t) * ks * sbt::kMfmaK);
        L.kA = take(sizeof(uint64_t) * ks * 64 * sbt::mfma_words(jp));
        L.xt = take(sizeof(float) * sbt::mfma_state_floats(n, M));  // x, y in the step's tiles
        L.yt = take(sizeof(float) * sbt::mfma_state_floats(n, M));
    }
    if (tiled && mode != SBT_DSB) {  // the tiled streaming step's plan
        const size_t nsuper = (static_cast<size_t>(n) + sbt::kTileSuper - 1) / sbt::kTileSuper;
        L.tile_info = take(2 * sizeof(int32_t) * nsuper * sbt::kTileSuper);
        L.tile_n = take(sizeof(int32_t) * nsuper);
        L.tile_cols = take(sizeof(int32_t) * pnnz);
        L.ploc = take(sizeof(uint16_t) * pnnz);
    }
    L.total = off;
    return L;
}

int check_params(const sbt_solve_params &p, const char *who) {
    if (!(p.a0 > 0.0) || !std::isfinite(p.a0))
        return fail(SBT_EINVAL, "%s: a0 must be finite and > 0", who);
    if (!(p.dt > 0.0) || !std::isfinite(p.dt))
        return fail(SBT_EINVAL, "%s: dt must be finite and > 0", who);
    if (std::isinf(p.c0)) return fail(SBT_EINVAL, "%s: c0 is infinite", who);
    if (p.agents < 1) return fail(SBT_EINVAL, "%s: agents must be >= 1", who);
    if (p.steps < 1) return fail(SBT_EINVAL, "%s: steps must be >= 1", who);
    if (p.energy_every < 0) return fail(SBT_EINVAL, "%s: energy_every must be >= 0", who);
    if (p.event < 0) return fail(SBT_EINVAL, "%s: event must be >= 0", who);
    if (p.kernel < SBT_KERNEL_AUTO || p.kernel > SBT_KERNEL_STREAM_MFMA)
        return fail(SBT_EINVAL, "%s: unknown kernel %d", who, p.kernel);
    if (p.tpb != 0 && p.tpb != 64 && p.tpb != 256 && p.tpb != 512 && p.tpb != 1024)
        return fail(SBT_EINVAL, "%s: tpb must be 0, 64, 256, 512 or 1024", who);
    if (p.precision < SBT_PREC_FP32 || p.precision > SBT_PREC_BF16X2)
        return fail(SBT_EINVAL, "%s: unknown precision %d", who, p.precision);
    if (p.reserved != 0) return fail(SBT_EINVAL, "%s: reserved must be 0", who);
    return SBT_OK;
}

int check_shape(int32_t n, int64_t nnz, int32_t M, const char *who) {
    if (n < 1) return fail(SBT_EINVAL, "%s: n must be >= 1", who);
    if (nnz < 0 || nnz + int64_t(sbt::kStreamChunk - 1) * n > std::numeric_limits<int32_t>::max())
        return fail(SBT_EINVAL, "%s: nnz %lld out of range", who, static_cast<long long>(nnz));
    if (static_cast<int64_t>(n) * M > (int64_t(1) << 31) - 1)
        return fail(SBT_EINVAL, "%s: n * agents exceeds 2^31 - 1", who);
    return SBT_OK;
}

int device_lds_limit() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 65536;
    return v;
}

// Resident-kernel shape, or tpb = 0 if no resident variant fits.
// Register-row variant when n <= kRegMaxN and the per-thread rows fit the
// register budget; otherwise the LDS-row variant while positions fit LDS.
sbt::ResidentShape resident_shape(int32_t n, int64_t nnz, int32_t max_row, int tpb_hint,
                                  int lds_limit) {
    sbt::ResidentShape S{0, 0, 0, 0, false, 0};
    auto pow2_at_least = [](int v) {
        int p = 1;
        while (p < v) p <<= 1;
        return p;
    };
    const bool hinted = tpb_hint == 64 || tpb_hint == 256 || tpb_hint == 512 || tpb_hint == 1024;
    // register-row variant: the fewest spins per thread whose workgroup
    // (a multiple of 64 threads) fits in 1024, or the hinted size
    if (n <= sbt::kRegMaxN) {
        for (const int spt : {1, 2, 3, 4, 8}) {
            const int tpb = ((n + spt - 1) / spt + 63) / 64 * 64;
            const int cap_tpb = hinted ? tpb_hint : 1024;
            if (tpb > cap_tpb) continue;
            const int maxtpb = tpb <= 256 ? 256 : (tpb <= 512 ? 512 : 1024);
            int rc = max_row <= 2 ? 2 : (max_row <= 4 ? 4 : 8), rr = 0;
            for (; rc >= 2; rc >>= 1) {
                if (sbt::reg_variant_fits(maxtpb, spt, rc, rc)) {
                    rr = rc;
                    break;
                }
                if (sbt::reg_variant_fits(maxtpb, spt, rc, 2)) {
                    rr = 2;
                    break;
                }
            }
            if (rr == 0) continue;
            const size_t lds =
                sizeof(float) * 2 * sbt::kRegStride + sizeof(double) * (maxtpb / 64) +
                (sizeof(int) + sizeof(float)) * sbt::kRegTailCap;
            if (lds > static_cast<size_t>(lds_limit)) break;
            S.tpb = tpb;
            S.spt = spt;
            S.rc = rc;
            S.rr = rr;
            S.lds_bytes = lds;
            return S;
        }
    }
    // LDS-row variant
    const int tpb = n <= 64 ? 64 : (n <= 1024 ? 256 : 1024);
    const int spt = pow2_at_least((n + tpb - 1) / tpb);
    if (spt > 16) return S;
    const size_t red = 16 + sizeof(double) * (tpb / 64);
    const size_t base = sizeof(float) * 2 * static_cast<size_t>(n) + red;
    const size_t jbytes = sizeof(int) * (static_cast<size_t>(n) + 1) +
                          (sizeof(int) + sizeof(float)) * static_cast<size_t>(nnz);
    if (base > static_cast<size_t>(lds_limit)) return S;
    S.tpb = tpb;
    S.spt = spt;
    S.rc = 0;
    S.jlds = base + jbytes <= static_cast<size_t>(lds_limit);
    S.lds_bytes = S.jlds ? base + jbytes : base;
    return S;
}

int pick_kernel(int32_t n, int64_t nnz, int32_t max_row, sbt_mode mode, const sbt_solve_params &p,
                int lds_limit,
                sbt::ResidentShape *shape) {
    sbt::ResidentShape S = resident_shape(n, nnz, max_row, p.tpb, lds_limit);
    if (shape) *shape = S;
    if (p.precision == SBT_PREC_FP16 || p.precision == SBT_PREC_BF16) {
        if (mode == SBT_DSB && (p.kernel == SBT_KERNEL_STREAM_MFMA ||
                                (p.kernel == SBT_KERNEL_AUTO && mfma_auto(mode, p.precision, n, p.agents))))
            return SBT_KERNEL_STREAM_MFMA;
        return fail(SBT_EUNSUPPORTED,
                    "16-bit couplings are solved by the batch functions (sbt_solve_batch) and, for "
                    "dSB, by the matrix-core streaming step");
    }
    const int stream_kind = SBT_KERNEL_STREAM;
    if (p.kernel == SBT_KERNEL_STREAM_TILE && mode == SBT_DSB)
        return fail(SBT_EUNSUPPORTED, "the tiled streaming step is for bSB and aSB (dSB reads "
                    "sign planes)");
    if (p.kernel == SBT_KERNEL_STREAM_MFMA) {
        if (mode != SBT_DSB)
            return fail(SBT_EUNSUPPORTED, "the matrix-core step is for dSB (bSB and aSB couple "
                        "through continuous positions)");
        return SBT_KERNEL_STREAM_MFMA;
    }
    if (p.precision == SBT_PREC_FP8 || p.precision == SBT_PREC_FP8_BLOCK ||
        p.precision == SBT_PREC_BF16X2) {
        if (p.kernel == SBT_KERNEL_RESIDENT)
            return fail(SBT_EUNSUPPORTED, "FP8 and BF16-pair coupling storage run on the streaming "
                        "kernel only");
        if (p.kernel == SBT_KERNEL_AUTO && mfma_auto(mode, p.precision, n, p.agents))
            return SBT_KERNEL_STREAM_MFMA;
        return p.kernel == SBT_KERNEL_AUTO ? stream_kind : p.kernel;
    }
    if (p.kernel == SBT_KERNEL_STREAM || p.kernel == SBT_KERNEL_STREAM_TILE ||
        p.kernel == SBT_KERNEL_STREAM_ROWS)
        return p.kernel;
    if (p.kernel == SBT_KERNEL_AUTO && mfma_auto(mode, p.precision, n, p.agents))
        return SBT_KERNEL_STREAM_MFMA;
    if (p.kernel == SBT_KERNEL_RESIDENT) {
        if (S.tpb == 0)
            return fail(SBT_EUNSUPPORTED, "resident kernel: n = %d does not fit in LDS", n);
        return SBT_KERNEL_RESIDENT;
    }
    // register-row residency wins whenever it fits; the LDS-row variant
    // only while there are too few agents to fill the streaming kernel's
    // 64-lane waves (measured: at 1024 agents and n = 8.5e3 streaming is
    // 2.6x faster)
    if (S.tpb != 0 && (S.rc > 0 || p.agents <= 128)) return SBT_KERNEL_RESIDENT;
    return stream_kind;
}

#define SBT_HIP(call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(SBT_EDEVICE, "%s: %s failed: %s", who, #call, hipGetErrorString(e_)); \
    } while (0)

}  // namespace

extern "C" void sbt_solve_params_default(sbt_solve_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->a0 = 1.0;
    p->dt = 1.0;
    p->c0 = 0.0;
    p->agents = 32;
    p->steps = 2000;
    p->seed = 0;
    p->event = 0;
    p->kernel = SBT_KERNEL_AUTO;
    p->energy_every = 0;
}

extern "C" size_t sbt_workspace_bytes(int32_t n, int64_t nnz, sbt_mode mode,
                                      const sbt_solve_params *p) {
    sbt::clear_error();
    if (!p) {
        fail(SBT_EINVAL, "sbt_workspace_bytes: params is NULL");
        return 0;
    }
    if (mode != SBT_BSB && mode != SBT_DSB && mode != SBT_ASB) {
        fail(SBT_EINVAL, "sbt_workspace_bytes: unknown mode");
        return 0;
    }
    if (check_params(*p, "sbt_workspace_bytes") != SBT_OK) return 0;
    if (check_shape(n, nnz, p->agents, "sbt_workspace_bytes") != SBT_OK) return 0;
    return make_layout(n, nnz, p->agents, p->steps, p->energy_every, mode, p->precision,
                       p->kernel).total;
}

extern "C" int sbt_select_kernel(int32_t n, int64_t nnz, int32_t max_row_nnz, sbt_mode mode,
                                 const sbt_solve_params *p) {
    sbt::clear_error();
    if (!p) return fail(SBT_EINVAL, "sbt_select_kernel: params is NULL");
    if (mode != SBT_BSB && mode != SBT_DSB && mode != SBT_ASB) return fail(SBT_EINVAL, "sbt_select_kernel: mode");
    int rc = check_params(*p, "sbt_select_kernel");
    if (rc) return rc;
    rc = check_shape(n, nnz, p->agents, "sbt_select_kernel");
    if (rc) return rc;
    if (max_row_nnz < 0) return fail(SBT_EINVAL, "sbt_select_kernel: max_row_nnz < 0");
    return pick_kernel(n, nnz, max_row_nnz, mode, *p, device_lds_limit(), nullptr);
}

extern "C" int sbt_solve_dev(const sbt_dev_qubo *q, int32_t max_row_nnz, sbt_mode mode,
                             const sbt_solve_params *p, void *workspace, size_t workspace_bytes,
                             const sbt_dev_result *out, void *stream) {
    const char *who = "sbt_solve_dev";
    sbt::clear_error();
    if (!q || !p || !out) return fail(SBT_EINVAL, "%s: NULL argument", who);
    if (mode != SBT_BSB && mode != SBT_DSB && mode != SBT_ASB) return fail(SBT_EINVAL, "%s: unknown mode", who);
    int rc = check_params(*p, who);
    if (rc) return rc;
    rc = check_shape(q->n, q->nnz, p->agents, who);
    if (rc) return rc;
    if (max_row_nnz < 0 || max_row_nnz > q->n)
        return fail(SBT_EINVAL, "%s: max_row_nnz %d out of range", who, max_row_nnz);
    if (!q->a || !q->row_ptr || (q->nnz > 0 && (!q->col || !q->b)))
        return fail(SBT_EINVAL, "%s: QUBO pointer is NULL", who);
    if (!out->T || !out->agent_energy || !out->best_energy || !out->best_agent)
        return fail(SBT_EINVAL, "%s: result pointer is NULL", who);
    const int32_t n = q->n, M = p->agents, K = p->steps;
    const int nnz = static_cast<int>(q->nnz);
    const Layout L = make_layout(n, q->nnz, M, K, p->energy_every, mode, p->precision, p->kernel);
    if (!workspace || workspace_bytes < L.total)
        return fail(SBT_EINVAL, "%s: workspace of %zu bytes is smaller than the %zu needed", who,
                    workspace_bytes, L.total);
    if ((out->trace || out->agent_trace) && L.n_ckpt == 0)
        return fail(SBT_EINVAL, "%s: trace requested but energy_every gives no checkpoint", who);

    sbt::ResidentShape shape;
    const int kernel = pick_kernel(n, q->nnz, max_row_nnz, mode, *p, device_lds_limit(), &shape);
    if (kernel < 0) return kernel;

    char *ws = static_cast<char *>(workspace);
    float *dJ = reinterpret_cast<float *>(ws + L.J);
    float *dh = reinterpret_cast<float *>(ws + L.h);
    double *scal = reinterpret_cast<double *>(ws + L.scal);
    double *prep = reinterpret_cast<double *>(ws + L.prep);
    int *perm = reinterpret_cast<int *>(ws + L.perm);
    float *sched = reinterpret_cast<float *>(ws + L.sched);
    float *xa = reinterpret_cast<float *>(ws + L.xa);
    float *xb = reinterpret_cast<float *>(ws + L.xb);
    float *dy = reinterpret_cast<float *>(ws + L.y);
    double *epart = reinterpret_cast<double *>(ws + L.epart);
    double *etrace = reinterpret_cast<double *>(ws + L.etrace);
    uint64_t *S0 = reinterpret_cast<uint64_t *>(ws + L.S0);
    uint64_t *S1 = reinterpret_cast<uint64_t *>(ws + L.S1);
    uint8_t *J8 = reinterpret_cast<uint8_t *>(ws + L.J8);
    float *rowscale = reinterpret_cast<float *>(ws + L.rowscale);
    int *prow = reinterpret_cast<int *>(ws + L.prow);
    int *pcol = reinterpret_cast<int *>(ws + L.pcol);
    float *pJ = reinterpret_cast<float *>(ws + L.pJ);
    hipStream_t st = static_cast<hipStream_t>(stream);

    const double c0_fixed = (std::isnan(p->c0) || p->c0 <= 0.0) ? 0.0 : p->c0;
    SBT_HIP(sbt::launch_prep(n, q->a, q->row_ptr, q->col, q->b, dJ, dh, prep, scal, c0_fixed, st));
    SBT_HIP(sbt::launch_init(n, M, p->seed, static_cast<uint32_t>(p->event), xa, dy, st));
    SBT_HIP(sbt::launch_schedule(K, p->a0, sched, st));

    const float dt = static_cast<float>(p->dt);
    const float dta0 = static_cast<float>(p->dt * p->a0);
    float *xfinal = xa;
    if (out->step_begin) SBT_HIP(hipEventRecord(static_cast<hipEvent_t>(out->step_begin), st));
    if (kernel == SBT_KERNEL_RESIDENT) {
        sbt::ResidentArgs A{};
        A.n = n;
        A.nnz = nnz;
        A.M = M;
        A.K = K;
        A.ckpt_every = p->energy_every;
        A.a0 = p->a0;
        A.dt = dt;
        A.dta0 = dta0;
        A.row_ptr = q->row_ptr;
        A.col = q->col;
        A.J = dJ;
        A.h = dh;
        A.scal = scal;
        A.a = q->a;
        A.b = q->b;
        A.x = xa;
        A.y = dy;
        A.etrace = etrace;
        A.perm = perm;
        A.sched = sched;
        if (shape.rc > 0) SBT_HIP(sbt::launch_row_order(n, q->row_ptr, perm, st));
        SBT_HIP(sbt::launch_resident(mode, A, shape, st));
    } else {
        sbt::StreamArgs A{};
        A.n = n;
        A.M = M;
        A.K = K;
        A.a0 = p->a0;
        A.dt = dt;
        A.dta0 = dta0;
        SBT_HIP(sbt::launch_stream_pack(n, q->row_ptr, q->col, dJ, prow, pcol, pJ, st));
        A.row_ptr = prow;
        A.col = pcol;
        A.J = pJ;
        A.h = dh;
        A.scal = scal;
        A.y = dy;
        A.sched = sched;
        A.sign_stride = sbt::stream_sign_stride(M);
        int jprec = sbt::kJFp32;
        const size_t pnnz = static_cast<size_t>(nnz) + (sbt::kStreamChunk - 1) * static_cast<size_t>(n);
        if (p->precision == SBT_PREC_FP8) {
            SBT_HIP(sbt::launch_quantize_fp8(n, prow, pJ, J8, rowscale, st));
            A.J8 = J8;
            A.rowscale = rowscale;
            jprec = sbt::kJFp8;
        } else if (p->precision == SBT_PREC_FP8_BLOCK) {
            // blocks are the padded rows' chunks of 8 (one scale per chunk load)
            float *blk = reinterpret_cast<float *>(ws + L.blkscale);
            SBT_HIP(sbt::launch_quantize_fp8_blocks(n, prow, static_cast<int64_t>(pnnz), pJ, J8, blk,
                                                    st));
            A.J8 = J8;
            A.blkscale = blk;
            jprec = sbt::kJFp8Blk;
        } else if (p->precision == SBT_PREC_BF16 || p->precision == SBT_PREC_FP16) {
            // the matrix-core step rounds the FP32 couplings itself
            jprec = p->precision == SBT_PREC_BF16 ? sbt::kJBf16 : sbt::kJFp16;
        } else if (p->precision == SBT_PREC_BF16X2) {
            uint32_t *J2 = reinterpret_cast<uint32_t *>(ws + L.J2);
            SBT_HIP(sbt::launch_split_bf16x2(n, prow, static_cast<int64_t>(pnnz), pJ, J2, st));
            A.J2 = J2;
            jprec = sbt::kJBf16x2;
        }
        const bool tiled = kernel == SBT_KERNEL_STREAM_TILE;
        sbt::TileArgs T{};
        if (tiled) {
            T.ucap = sbt::kTileColsDefault;
            T.tile_info = reinterpret_cast<int2 *>(ws + L.tile_info);
            T.tile_n = reinterpret_cast<int *>(ws + L.tile_n);
            T.tile_cols = reinterpret_cast<int *>(ws + L.tile_cols);
            T.ploc = reinterpret_cast<uint16_t *>(ws + L.ploc);
            SBT_HIP(sbt::launch_tile_plan(n, prow, pcol, T, st));
        }
        const bool mfma = kernel == SBT_KERNEL_STREAM_MFMA;
        sbt::MfmaArgs P{};
        if (mfma) {
            P.kcnt = reinterpret_cast<int *>(ws + L.kcnt);
            P.koff = reinterpret_cast<int *>(ws + L.koff);
            P.kcol = reinterpret_cast<int *>(ws + L.kcol);
            P.kA = reinterpret_cast<uint64_t *>(ws + L.kA);
            SBT_HIP(sbt::launch_mfma_plan(jprec, A, P, st));
        }
        const bool quads = kernel == SBT_KERNEL_STREAM && quad_step(mode, M);
        sbt::QuadArgs Q{};
        if (quads) {
            Q.qcnt = reinterpret_cast<int *>(ws + L.qcnt);
            Q.qoff = reinterpret_cast<int *>(ws + L.qoff);
            Q.qcol = reinterpret_cast<int *>(ws + L.qcol);
            Q.qJ = reinterpret_cast<float *>(ws + L.qJ);
            SBT_HIP(sbt::launch_quad_plan(jprec, A, Q, st));
        }
        // dSB: x, y in place, signs ping-pong between S0 and S1;
        // bSB: positions ping-pong between xa and xb
        float *xin = xa, *xout = xb;
        uint64_t *Sin = S0, *Sout = S1;
        float *xt = reinterpret_cast<float *>(ws + L.xt), *yt = reinterpret_cast<float *>(ws + L.yt);
        if (mfma) {
            SBT_HIP(sbt::launch_mfma_signs(n, M, xa, reinterpret_cast<uint8_t *>(S0), st));
            SBT_HIP(sbt::launch_mfma_state(n, M, true, xa, xt, st));
            SBT_HIP(sbt::launch_mfma_state(n, M, true, dy, yt, st));
        } else if (mode == SBT_DSB)
            SBT_HIP(sbt::launch_sign_planes(n, M, xa, S0, st));
        int ck = 0;
        for (int k = 0; k < K; ++k) {
            if (tiled)
                SBT_HIP(sbt::launch_stream_tile(static_cast<int>(mode), jprec, A, T, k, xin, xout, st));
            else if (mfma)
                SBT_HIP(sbt::launch_stream_mfma(jprec, A, P, k, xt, yt, reinterpret_cast<const uint8_t *>(Sin),
                                                reinterpret_cast<uint8_t *>(Sout), st));
            else if (quads)
                SBT_HIP(sbt::launch_stream_quad(static_cast<int>(mode), A, Q, k, xin, xout, st));
            else
                SBT_HIP(sbt::launch_stream2(static_cast<int>(mode), jprec, A, k, xin, xout, Sin, Sout, st));
            std::swap(xin, xout);
            std::swap(Sin, Sout);
            if (p->energy_every > 0 && (k + 1) % p->energy_every == 0) {
                if (mfma) SBT_HIP(sbt::launch_mfma_state(n, M, false, xt, xin, st));  // xin == xa (dSB)
                SBT_HIP(sbt::launch_energy(n, M, q->a, q->row_ptr, q->col, q->b, xin, epart,
                                           etrace + static_cast<size_t>(ck) * M, st));
                ++ck;
            }
        }
        if (mfma) {
            SBT_HIP(sbt::launch_mfma_state(n, M, false, xt, xin, st));
            SBT_HIP(sbt::launch_mfma_state(n, M, false, yt, dy, st));
        }
        xfinal = xin;
    }
    if (out->step_end) SBT_HIP(hipEventRecord(static_cast<hipEvent_t>(out->step_end), st));
    SBT_HIP(sbt::launch_energy(n, M, q->a, q->row_ptr, q->col, q->b, xfinal, epart,
                               out->agent_energy, st));
    SBT_HIP(sbt::launch_select_best(n, M, out->agent_energy, xfinal, out->best_energy,
                                    out->best_agent, out->T, st));
    if (out->trace) SBT_HIP(sbt::launch_trace_reduce(L.n_ckpt, M, etrace, out->trace, st));
    if (out->agent_trace)
        SBT_HIP(hipMemcpyAsync(out->agent_trace, etrace, sizeof(double) * L.n_ckpt * M,
                               hipMemcpyDeviceToDevice, st));
    const size_t nm = static_cast<size_t>(n) * M;
    if (out->x_final)
        SBT_HIP(hipMemcpyAsync(out->x_final, xfinal, nm * sizeof(float), hipMemcpyDeviceToDevice, st));
    if (out->y_final)
        SBT_HIP(hipMemcpyAsync(out->y_final, dy, nm * sizeof(float), hipMemcpyDeviceToDevice, st));
    if (out->scalars)
        SBT_HIP(hipMemcpyAsync(out->scalars, scal, 4 * sizeof(double), hipMemcpyDeviceToDevice, st));
    return SBT_OK;
}

// ----------------------------------------------------------- host solve

namespace {

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

struct HostStream {
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~HostStream() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (s) (void)hipStreamDestroy(s);
    }
};

}  // namespace

extern "C" int sbt_solve(const sbt_qubo *q, sbt_mode mode, const sbt_solve_params *pp,
                         sbt_result *out) {
    const char *who = "sbt_solve";
    sbt::clear_error();
    if (!out) return fail(SBT_EINVAL, "%s: result is NULL", who);
    sbt_solve_params p;
    if (pp)
        p = *pp;
    else
        sbt_solve_params_default(&p);
    if (mode != SBT_BSB && mode != SBT_DSB && mode != SBT_ASB) return fail(SBT_EINVAL, "%s: unknown mode", who);
    int rc = check_params(p, who);
    if (rc) return rc;
    int32_t max_row = 0;
    rc = sbt::validate_qubo_host(q, who, "qubo", &max_row);
    if (rc) return rc;
    rc = check_shape(q->n, q->nnz, p.agents, who);
    if (rc) return rc;
    const int32_t n = q->n, M = p.agents;
    const int64_t nnz = q->nnz;
    const int n_ckpt = p.energy_every > 0 ? p.steps / p.energy_every : 0;
    if ((out->trace || out->agent_trace) && n_ckpt == 0)
        return fail(SBT_EINVAL, "%s: trace requested but energy_every gives no checkpoint", who);

    std::vector<int32_t> rp32(n + 1);
    for (int32_t i = 0; i <= n; ++i) rp32[i] = static_cast<int32_t>(q->row_ptr[i]);
    const size_t ws_bytes =
        make_layout(n, nnz, M, p.steps, p.energy_every, mode, p.precision, p.kernel).total;
    const size_t nm = static_cast<size_t>(n) * M;

    DevBuf da, drp, dcol, db, dws, dT, dE, dbe, dbm, dsc, dx, dy, dtr, dat;
    auto alloc = [&](DevBuf &b, size_t bytes) {
        return hipMalloc(&b.p, std::max<size_t>(bytes, 1));
    };
    if (alloc(da, sizeof(double) * n) != hipSuccess || alloc(drp, sizeof(int32_t) * (n + 1)) ||
        alloc(dcol, sizeof(int32_t) * nnz) || alloc(db, sizeof(double) * nnz) ||
        alloc(dws, ws_bytes) || alloc(dT, n) || alloc(dE, sizeof(double) * M) ||
        alloc(dbe, sizeof(double)) || alloc(dbm, sizeof(int32_t)) || alloc(dsc, 4 * sizeof(double)) ||
        (out->x_final && alloc(dx, sizeof(float) * nm)) ||
        (out->y_final && alloc(dy, sizeof(float) * nm)) ||
        (out->trace && alloc(dtr, sizeof(double) * n_ckpt)) ||
        (out->agent_trace && alloc(dat, sizeof(double) * n_ckpt * M)))
        return fail(SBT_ENOMEM, "%s: device allocation failed", who);
    HostStream hs;
    SBT_HIP(hipStreamCreateWithFlags(&hs.s, hipStreamNonBlocking));
    SBT_HIP(hipEventCreate(&hs.e0));
    SBT_HIP(hipEventCreate(&hs.e1));
    SBT_HIP(hipMemcpyAsync(da.p, q->a, sizeof(double) * n, hipMemcpyHostToDevice, hs.s));
    SBT_HIP(hipMemcpyAsync(drp.p, rp32.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, hs.s));
    if (nnz > 0) {
        SBT_HIP(hipMemcpyAsync(dcol.p, q->col, sizeof(int32_t) * nnz, hipMemcpyHostToDevice, hs.s));
        SBT_HIP(hipMemcpyAsync(db.p, q->b, sizeof(double) * nnz, hipMemcpyHostToDevice, hs.s));
    }
    sbt_dev_qubo dq{n, nnz, static_cast<const double *>(da.p), static_cast<const int32_t *>(drp.p),
                    static_cast<const int32_t *>(dcol.p), static_cast<const double *>(db.p)};
    sbt_dev_result dr{};
    dr.T = static_cast<int8_t *>(dT.p);
    dr.agent_energy = static_cast<double *>(dE.p);
    dr.best_energy = static_cast<double *>(dbe.p);
    dr.best_agent = static_cast<int32_t *>(dbm.p);
    dr.scalars = static_cast<double *>(dsc.p);
    dr.x_final = static_cast<float *>(dx.p);
    dr.y_final = static_cast<float *>(dy.p);
    dr.trace = static_cast<double *>(dtr.p);
    dr.agent_trace = static_cast<double *>(dat.p);
    const int kernel = pick_kernel(n, nnz, max_row, mode, p, device_lds_limit(), nullptr);
    if (kernel < 0) return kernel;
    SBT_HIP(hipEventRecord(hs.e0, hs.s));
    rc = sbt_solve_dev(&dq, max_row, mode, &p, dws.p, ws_bytes, &dr, hs.s);
    if (rc) return rc;
    SBT_HIP(hipEventRecord(hs.e1, hs.s));
    double scal[4];
    int32_t bm = 0;
    SBT_HIP(hipMemcpyAsync(&out->energy, dbe.p, sizeof(double), hipMemcpyDeviceToHost, hs.s));
    SBT_HIP(hipMemcpyAsync(&bm, dbm.p, sizeof(int32_t), hipMemcpyDeviceToHost, hs.s));
    SBT_HIP(hipMemcpyAsync(scal, dsc.p, sizeof scal, hipMemcpyDeviceToHost, hs.s));
    if (out->T) SBT_HIP(hipMemcpyAsync(out->T, dT.p, n, hipMemcpyDeviceToHost, hs.s));
    if (out->agent_energy)
        SBT_HIP(hipMemcpyAsync(out->agent_energy, dE.p, sizeof(double) * M, hipMemcpyDeviceToHost, hs.s));
    if (out->x_final)
        SBT_HIP(hipMemcpyAsync(out->x_final, dx.p, sizeof(float) * nm, hipMemcpyDeviceToHost, hs.s));
    if (out->y_final)
        SBT_HIP(hipMemcpyAsync(out->y_final, dy.p, sizeof(float) * nm, hipMemcpyDeviceToHost, hs.s));
    if (out->trace)
        SBT_HIP(hipMemcpyAsync(out->trace, dtr.p, sizeof(double) * n_ckpt, hipMemcpyDeviceToHost, hs.s));
    if (out->agent_trace)
        SBT_HIP(hipMemcpyAsync(out->agent_trace, dat.p, sizeof(double) * n_ckpt * M,
                               hipMemcpyDeviceToHost, hs.s));
    SBT_HIP(hipStreamSynchronize(hs.s));
    float ms = 0.0f;
    SBT_HIP(hipEventElapsedTime(&ms, hs.e0, hs.e1));
    out->best_agent = bm;
    out->c0 = scal[0];
    out->ising_offset = scal[1];
    out->kernel_used = kernel;
    out->elapsed_s = 1e-3 * ms;
    out->trace_len = n_ckpt;
    return SBT_OK;
}
