// Host side of the batched solver: workspace layout, the work-item
// schedule, and the sbt_batch_* / sbt_solve_batch entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>

#include "common.hpp"
#include "sb_kernels.hpp"
#include "sbtrack.h"

namespace {

using sbt::fail;

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Schedule {
    std::vector<sbt::BatchEvent> ev;
    // items of the 1024-thread launch first, then those of the 512-thread
    // launch, each group in decreasing-cost order
    std::vector<int32_t> item_event, item_agent0;
    int n_large = 0, n_small = 0;  // items per launch
    int64_t sum_n = 0, sum_nnz = 0;
    // events above the band limit: one gang of row bands per agent
    std::vector<sbt::GangDesc> gangs;
    std::vector<int32_t> gitem_gang, gitem_band;
    int64_t xg_floats = 0, part_entries = 0;
    int max_bands = 0;
    int items() const { return static_cast<int>(item_event.size() + gitem_gang.size()); }
};

int tpb_of(bool small) { return small ? sbt::kBatchTPBSmall : sbt::kBatchTPB; }

// Agents per work item: the largest power of two A with n * A within
// `fill` of the shape's slots (and A <= agents, A <= its threads); at least
// one agent.
int lg_agents_for(int32_t n, int32_t M, int tpb, double fill) {
    const double cap = fill * tpb * sbt::kBatchSPT;
    int lg = 0;
    while ((2 << lg) <= M && (2 << lg) <= tpb && static_cast<double>(n) * (2 << lg) <= cap) ++lg;
    return lg;
}

int check_tuning(const sbt_batch_tuning &t, const char *who) {
    if (t.split_n < 0) return fail(SBT_EINVAL, "%s: tuning split_n must be >= 0", who);
    if (t.tail_words < 0 || t.tail_words > sbt::kBatchTailCap)
        return fail(SBT_EINVAL, "%s: tuning tail_words must be in [0, %d]", who, sbt::kBatchTailCap);
    if (!(t.fill > 0.0) || !(t.fill <= 1.0))
        return fail(SBT_EINVAL, "%s: tuning fill must be in (0, 1]", who);
    if (t.band_rows < 0 || t.band_rows > sbt::kBatchSlots)
        return fail(SBT_EINVAL, "%s: tuning band_rows must be in [0, %d]", who, sbt::kBatchSlots);
    if (t.reserved != 0) return fail(SBT_EINVAL, "%s: tuning reserved must be 0", who);
    return SBT_OK;
}

int make_schedule(const int32_t *n, const int64_t *nnz, int32_t E, const double *c0_scale,
                  int32_t same_start, const sbt_solve_params &p, const sbt_batch_tuning &tu,
                  Schedule &S, const char *who) {
    if (E < 1) return fail(SBT_EINVAL, "%s: n_events must be >= 1", who);
    if (!n || !nnz) return fail(SBT_EINVAL, "%s: n or nnz is NULL", who);
    int rc = check_tuning(tu, who);
    if (rc) return rc;
    if (c0_scale)
        for (int32_t e = 0; e < E; ++e)
            if (!(c0_scale[e] > 0.0) || !std::isfinite(c0_scale[e]))
                return fail(SBT_EINVAL, "%s: c0_scale[%d] must be finite and > 0", who, e);
    S.ev.resize(E);
    struct Item {
        int64_t cost;
        int32_t e, a0;
    };
    std::vector<Item> items[2];  // [0]: 1024-thread shape, [1]: 512-thread shape
    const int band_limit = tu.band_rows > 0 ? tu.band_rows : sbt::kBatchSlots;
    const int n_ckpt = p.energy_every > 0 ? p.steps / p.energy_every : 0;
    S.gangs.clear();
    S.xg_floats = S.part_entries = 0;
    S.max_bands = 0;
    std::vector<int64_t> gang_cost;
    int64_t row_off = 0, nz_off = 0;
    for (int32_t e = 0; e < E; ++e) {
        if (n[e] < 1) return fail(SBT_EINVAL, "%s: event %d has n = %d", who, e, n[e]);
        if (nnz[e] < 0) return fail(SBT_EINVAL, "%s: event %d has nnz < 0", who, e);
        const bool small = n[e] <= tu.split_n && n[e] <= sbt::kBatchSlotsSmall;
        sbt::BatchEvent &d = S.ev[e];
        d.n = n[e];
        d.nnz = static_cast<int>(nnz[e]);
        d.row_off = static_cast<int>(row_off);
        d.rp_off = static_cast<int>(row_off + e);
        d.nz_off = static_cast<int>(nz_off);
        d.lg_agents = lg_agents_for(n[e], p.agents, tpb_of(small), tu.fill);
        d.event_id = same_start ? p.event : p.event + e;
        d.c0_scale = c0_scale ? static_cast<float>(c0_scale[e]) : 1.0f;
        if (n[e] > band_limit) {
            // row bands of balanced size, one gang per agent
            const int bands = (n[e] + band_limit - 1) / band_limit;
            const int rows = (n[e] + bands - 1) / bands;
            S.max_bands = std::max(S.max_bands, bands);
            for (int a = 0; a < p.agents; ++a) {
                sbt::GangDesc gd{};
                gd.e = e;
                gd.agent = a;
                gd.bands = bands;
                gd.rows = rows;
                gd.x_off = S.xg_floats;
                gd.part_off = static_cast<int>(S.part_entries);
                S.gangs.push_back(gd);
                gang_cost.push_back(static_cast<int64_t>(n[e]) + nnz[e]);
                S.xg_floats += 2 * static_cast<int64_t>(n[e]);
                S.part_entries += static_cast<int64_t>(bands) * (n_ckpt + 1);
            }
            if (S.part_entries > INT32_MAX / 2)
                return fail(SBT_EINVAL, "%s: too many row bands for 32-bit offsets", who);
        } else {
            const int A = 1 << d.lg_agents;
            for (int a0 = 0; a0 < p.agents; a0 += A) {
                const int used = std::min(A, p.agents - a0);
                items[small ? 1 : 0].push_back({(static_cast<int64_t>(n[e]) + nnz[e]) * used, e, a0});
            }
        }
        row_off += n[e];
        nz_off += nnz[e];
        if (row_off + e + 1 > INT32_MAX / 2 || nz_off > INT32_MAX / 2)
            return fail(SBT_EINVAL, "%s: batch too large for 32-bit offsets", who);
    }
    S.item_event.clear();
    S.item_agent0.clear();
    for (auto &v : items) {
        // longest items first (ties: event, then agent order)
        std::stable_sort(v.begin(), v.end(),
                         [](const Item &l, const Item &r) { return l.cost > r.cost; });
        for (const Item &it : v) {
            S.item_event.push_back(it.e);
            S.item_agent0.push_back(it.a0);
        }
    }
    S.n_large = static_cast<int>(items[0].size());
    S.n_small = static_cast<int>(items[1].size());
    // gangs: largest events first, then agent order; items gang after gang
    std::vector<int> order(S.gangs.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int l, int r) { return gang_cost[l] > gang_cost[r]; });
    std::vector<sbt::GangDesc> sorted;
    sorted.reserve(order.size());
    for (int g : order) sorted.push_back(S.gangs[g]);
    S.gangs.swap(sorted);
    S.gitem_gang.clear();
    S.gitem_band.clear();
    for (size_t g = 0; g < S.gangs.size(); ++g)
        for (int b = 0; b < S.gangs[g].bands; ++b) {
            S.gitem_gang.push_back(static_cast<int32_t>(g));
            S.gitem_band.push_back(b);
        }
    S.sum_n = row_off;
    S.sum_nnz = nz_off;
    return SBT_OK;
}

struct BatchLayout {
    size_t ev, item_e, item_a, J16, h, c0, offset, perm, sched, counter, etrace, energy, T;
    size_t gangs, gitem_g, gitem_b, xg, gints, gpart, gclock, done;
    size_t total;
    int n_ckpt;
};

BatchLayout make_layout(const Schedule &S, const sbt_solve_params &p) {
    BatchLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + std::max<size_t>(bytes, 1));
        return at;
    };
    const size_t E = S.ev.size(), I = S.item_event.size(), M = static_cast<size_t>(p.agents);
    L.n_ckpt = p.energy_every > 0 ? p.steps / p.energy_every : 0;
    L.ev = take(sizeof(sbt::BatchEvent) * E);
    L.item_e = take(sizeof(int32_t) * I);
    L.item_a = take(sizeof(int32_t) * I);
    L.J16 = take(sizeof(uint16_t) * static_cast<size_t>(S.sum_nnz));
    L.h = take(sizeof(float) * static_cast<size_t>(S.sum_n));
    L.c0 = take(sizeof(float) * E);
    L.offset = take(sizeof(double) * E);
    L.perm = take(sizeof(int32_t) * static_cast<size_t>(S.sum_n));
    L.sched = take(sizeof(float) * static_cast<size_t>(p.steps));
    L.counter = take(2 * sizeof(int32_t));  // one per launch
    L.etrace = take(sizeof(double) * E * static_cast<size_t>(L.n_ckpt) * M);
    L.energy = take(sizeof(double) * E * M);
    L.T = take(static_cast<size_t>(S.sum_n) * M);
    const size_t G = S.gangs.size(), GI = S.gitem_gang.size();
    L.gangs = take(sizeof(sbt::GangDesc) * G);
    L.gitem_g = take(sizeof(int32_t) * GI);
    L.gitem_b = take(sizeof(int32_t) * GI);
    L.xg = take(sizeof(float) * static_cast<size_t>(S.xg_floats));
    L.gints = take(sizeof(int32_t) * (G + 2));  // arrivals per gang, fault flag, queue
    L.gpart = take(sizeof(double) * static_cast<size_t>(S.part_entries));
    L.gclock = take(sizeof(int64_t) * static_cast<size_t>(S.part_entries));
    L.done = take(sizeof(int32_t) * E);  // events whose target was reached
    L.total = off;
    return L;
}

int check_batch_params(const sbt_solve_params &p, const char *who) {
    if (!(p.a0 > 0.0) || !std::isfinite(p.a0) || !(p.dt > 0.0) || !std::isfinite(p.dt))
        return fail(SBT_EINVAL, "%s: a0 and dt must be finite and > 0", who);
    if (std::isinf(p.c0)) return fail(SBT_EINVAL, "%s: c0 is infinite", who);
    if (p.agents < 1 || p.steps < 1 || p.energy_every < 0 || p.event < 0)
        return fail(SBT_EINVAL, "%s: invalid agents, steps, energy_every or event", who);
    return SBT_OK;
}

int cu_count() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 256;
    return v > 0 ? v : 256;
}

#define SBT_HIP(call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(SBT_EDEVICE, "%s: %s failed: %s", who, #call, hipGetErrorString(e_)); \
    } while (0)

}  // namespace

extern "C" void sbt_batch_tuning_default(sbt_batch_tuning *t) {
    if (!t) return;
    std::memset(t, 0, sizeof *t);
    t->split_n = 0;
    t->tail_words = sbt::kBatchTailCap;
    t->fill = 1.0;
}

namespace {

sbt_batch_tuning tuning_or_default(const sbt_batch_tuning *t) {
    sbt_batch_tuning d;
    sbt_batch_tuning_default(&d);
    if (!t) return d;
    sbt_batch_tuning r = *t;
    r.from_cache = 0;
    return r;
}

}  // namespace

extern "C" size_t sbt_batch_workspace_bytes_tuned(const int32_t *n, const int64_t *nnz,
                                                  int32_t n_events, const sbt_solve_params *p,
                                                  const sbt_batch_tuning *t) {
    sbt::clear_error();
    const char *who = "sbt_batch_workspace_bytes";
    if (!p) {
        fail(SBT_EINVAL, "%s: params is NULL", who);
        return 0;
    }
    if (check_batch_params(*p, who)) return 0;
    Schedule S;
    if (make_schedule(n, nnz, n_events, nullptr, 0, *p, tuning_or_default(t), S, who)) return 0;
    return make_layout(S, *p).total;
}

extern "C" size_t sbt_batch_workspace_bytes(const int32_t *n, const int64_t *nnz, int32_t n_events,
                                            const sbt_solve_params *p) {
    return sbt_batch_workspace_bytes_tuned(n, nnz, n_events, p, nullptr);
}

extern "C" int sbt_batch_plan_tuned(const int32_t *n, const int64_t *nnz, int32_t n_events,
                                    const double *c0_scale, int32_t same_start,
                                    const sbt_solve_params *p, const sbt_batch_tuning *t,
                                    void *workspace, size_t workspace_bytes, void *stream) {
    const char *who = "sbt_batch_plan";
    sbt::clear_error();
    if (!p) return fail(SBT_EINVAL, "%s: params is NULL", who);
    int rc = check_batch_params(*p, who);
    if (rc) return rc;
    Schedule S;
    rc = make_schedule(n, nnz, n_events, c0_scale, same_start, *p, tuning_or_default(t), S, who);
    if (rc) return rc;
    const BatchLayout L = make_layout(S, *p);
    if (!workspace || workspace_bytes < L.total)
        return fail(SBT_EINVAL, "%s: workspace of %zu bytes is smaller than the %zu needed", who,
                    workspace_bytes, L.total);
    char *ws = static_cast<char *>(workspace);
    hipStream_t st = static_cast<hipStream_t>(stream);
    SBT_HIP(hipMemcpyAsync(ws + L.ev, S.ev.data(), sizeof(sbt::BatchEvent) * S.ev.size(),
                           hipMemcpyHostToDevice, st));
    SBT_HIP(hipMemcpyAsync(ws + L.item_e, S.item_event.data(), sizeof(int32_t) * S.item_event.size(),
                           hipMemcpyHostToDevice, st));
    SBT_HIP(hipMemcpyAsync(ws + L.item_a, S.item_agent0.data(),
                           sizeof(int32_t) * S.item_agent0.size(), hipMemcpyHostToDevice, st));
    if (!S.gangs.empty()) {
        if (S.max_bands > cu_count())
            return fail(SBT_EUNSUPPORTED, "%s: an event needs %d row bands at once, more than the "
                        "device's %d CUs", who, S.max_bands, cu_count());
        SBT_HIP(hipMemcpyAsync(ws + L.gangs, S.gangs.data(), sizeof(sbt::GangDesc) * S.gangs.size(),
                               hipMemcpyHostToDevice, st));
        SBT_HIP(hipMemcpyAsync(ws + L.gitem_g, S.gitem_gang.data(),
                               sizeof(int32_t) * S.gitem_gang.size(), hipMemcpyHostToDevice, st));
        SBT_HIP(hipMemcpyAsync(ws + L.gitem_b, S.gitem_band.data(),
                               sizeof(int32_t) * S.gitem_band.size(), hipMemcpyHostToDevice, st));
    }
    SBT_HIP(hipStreamSynchronize(st));
    return S.items();
}

extern "C" int sbt_batch_plan(const int32_t *n, const int64_t *nnz, int32_t n_events,
                              const double *c0_scale, int32_t same_start,
                              const sbt_solve_params *p, void *workspace, size_t workspace_bytes,
                              void *stream) {
    return sbt_batch_plan_tuned(n, nnz, n_events, c0_scale, same_start, p, nullptr, workspace,
                                workspace_bytes, stream);
}

extern "C" int sbt_batch_run_tuned(const sbt_dev_batch *batch, sbt_mode mode, sbt_precision prec,
                                   const sbt_solve_params *p, const sbt_batch_tuning *t,
                                   void *workspace, size_t workspace_bytes,
                                   const sbt_dev_batch_result *out, void *stream) {
    const char *who = "sbt_batch_run";
    sbt::clear_error();
    if (!batch || !p || !out) return fail(SBT_EINVAL, "%s: NULL argument", who);
    if (mode != SBT_BSB && mode != SBT_DSB && mode != SBT_ASB)
        return fail(SBT_EINVAL, "%s: unknown mode", who);
    if (prec != SBT_PREC_FP16 && prec != SBT_PREC_BF16)
        return fail(SBT_EUNSUPPORTED, "%s: batches hold 16-bit couplings (FP16 or BF16)", who);
    int rc = check_batch_params(*p, who);
    if (rc) return rc;
    const sbt_batch_tuning tu = tuning_or_default(t);
    Schedule S;
    rc = make_schedule(batch->n, batch->nnz, batch->n_events, nullptr, 0, *p, tu, S, who);
    if (rc) return rc;
    const BatchLayout L = make_layout(S, *p);
    if (!workspace || workspace_bytes < L.total)
        return fail(SBT_EINVAL, "%s: workspace of %zu bytes is smaller than the %zu needed", who,
                    workspace_bytes, L.total);
    if (!batch->a || !batch->row_ptr || (S.sum_nnz > 0 && (!batch->col || !batch->b)))
        return fail(SBT_EINVAL, "%s: batch array is NULL", who);
    if (!out->best_energy || !out->best_agent || !out->best_T)
        return fail(SBT_EINVAL, "%s: result pointer is NULL", who);
    if ((out->trace || out->agent_trace) && L.n_ckpt == 0)
        return fail(SBT_EINVAL, "%s: trace requested but energy_every gives no checkpoint", who);
    char *ws = static_cast<char *>(workspace);
    hipStream_t st = static_cast<hipStream_t>(stream);

    sbt::BatchArgs B{};
    B.E = batch->n_events;
    B.M = p->agents;
    B.K = p->steps;
    B.tail_cap = tu.tail_words;
    B.ckpt_every = p->energy_every;
    B.n_ckpt = L.n_ckpt;
    B.seed_lo = static_cast<uint32_t>(p->seed & 0xffffffffu);
    B.seed_hi = static_cast<uint32_t>(p->seed >> 32);
    B.dt = static_cast<float>(p->dt);
    B.dta0 = static_cast<float>(p->dt * p->a0);
    B.c0_fixed = (std::isnan(p->c0) || p->c0 <= 0.0) ? 0.0 : p->c0;
    B.ev = reinterpret_cast<const sbt::BatchEvent *>(ws + L.ev);
    B.item_event = reinterpret_cast<const int *>(ws + L.item_e);
    B.item_agent0 = reinterpret_cast<const int *>(ws + L.item_a);
    B.row_ptr = batch->row_ptr;
    B.col = batch->col;
    B.a = batch->a;
    B.b = batch->b;
    B.J16 = reinterpret_cast<uint16_t *>(ws + L.J16);
    B.h = reinterpret_cast<float *>(ws + L.h);
    B.c0 = reinterpret_cast<float *>(ws + L.c0);
    B.offset = out->offset ? out->offset : reinterpret_cast<double *>(ws + L.offset);
    B.perm = reinterpret_cast<int *>(ws + L.perm);
    B.sched = reinterpret_cast<const float *>(ws + L.sched);
    B.etrace = reinterpret_cast<double *>(ws + L.etrace);
    B.energy = out->agent_energy ? out->agent_energy : reinterpret_cast<double *>(ws + L.energy);
    B.trace = out->trace;
    B.best_energy = out->best_energy;
    B.best_agent = out->best_agent;
    B.T = out->agent_T ? out->agent_T : reinterpret_cast<int8_t *>(ws + L.T);
    B.x_out = out->agent_x;
    B.best_T = out->best_T;
    B.ckpt_clock = reinterpret_cast<long long *>(out->ckpt_clock);
    int *counters = reinterpret_cast<int *>(ws + L.counter);
    if (batch->target) {
        if (L.n_ckpt == 0)
            return fail(SBT_EINVAL, "%s: a target needs checkpoints (energy_every > 0)", who);
        B.target = batch->target;
        B.done = reinterpret_cast<int *>(ws + L.done);
    }

    SBT_HIP(sbt::launch_schedule(p->steps, p->a0, reinterpret_cast<float *>(ws + L.sched), st));
    const int jprec = prec == SBT_PREC_FP16 ? sbt::kJFp16 : sbt::kJBf16;
    const int cus = cu_count();
    hipError_t e = sbt::launch_batch_prep(jprec, B, st);
    if (e != hipSuccess) return fail(SBT_EDEVICE, "%s: batch prep: %s", who, hipGetErrorString(e));
    SBT_HIP(sbt::launch_batch_reset(counters, 2, st));
    if (B.done) SBT_HIP(sbt::launch_zero_ints(B.done, batch->n_events, st));
    const int n_gangs = static_cast<int>(S.gangs.size());
    if (n_gangs > 0) {
        if (S.max_bands > cus)
            return fail(SBT_EUNSUPPORTED, "%s: an event needs %d row bands at once, more than the "
                        "device's %d CUs", who, S.max_bands, cus);
        int *gints = reinterpret_cast<int *>(ws + L.gints);
        SBT_HIP(sbt::launch_zero_ints(gints, n_gangs + 2, st));
        B.gang_items = static_cast<int>(S.gitem_gang.size());
        B.gitem_gang = reinterpret_cast<const int *>(ws + L.gitem_g);
        B.gitem_band = reinterpret_cast<const int *>(ws + L.gitem_b);
        B.gangs = reinterpret_cast<const sbt::GangDesc *>(ws + L.gangs);
        B.xg = reinterpret_cast<float *>(ws + L.xg);
        B.arrive = gints;
        B.gang_fault = gints + n_gangs;
        B.gang_counter = gints + n_gangs + 1;
        B.gpart = reinterpret_cast<double *>(ws + L.gpart);
        B.gclock = reinterpret_cast<long long *>(ws + L.gclock);
    }
    if (out->step_begin) SBT_HIP(hipEventRecord(static_cast<hipEvent_t>(out->step_begin), st));
    // gangs of row bands first (the largest events), on a persistent grid at
    // least as large as any gang
    if (n_gangs > 0) {
        sbt::BatchArgs LG = B;
        LG.grid = std::min(B.gang_items, cus);
        e = sbt::launch_batch_gang(static_cast<int>(mode), jprec, LG, st);
        if (e != hipSuccess) return fail(SBT_EDEVICE, "%s: gang kernel: %s", who, hipGetErrorString(e));
    }
    // the 1024-thread items (one workgroup per CU), then the 512-thread items
    // (two per CU), each launch a persistent grid over its own queue
    if (S.n_large > 0) {
        sbt::BatchArgs L0 = B;
        L0.item_begin = 0;
        L0.n_items = S.n_large;
        L0.counter = counters;
        L0.grid = std::min(S.n_large, cus);
        e = sbt::launch_batch_steps(static_cast<int>(mode), jprec, sbt::kBatchTPB, L0, st);
        if (e != hipSuccess) return fail(SBT_EDEVICE, "%s: batch kernel: %s", who, hipGetErrorString(e));
    }
    if (S.n_small > 0) {
        sbt::BatchArgs L1 = B;
        L1.item_begin = S.n_large;
        L1.n_items = S.n_small;
        L1.counter = counters + 1;
        L1.grid = std::min(S.n_small, 2 * cus);
        e = sbt::launch_batch_steps(static_cast<int>(mode), jprec, sbt::kBatchTPBSmall, L1, st);
        if (e != hipSuccess) return fail(SBT_EDEVICE, "%s: batch kernel: %s", who, hipGetErrorString(e));
    }
    if (out->step_end) SBT_HIP(hipEventRecord(static_cast<hipEvent_t>(out->step_end), st));
    if (n_gangs > 0) {
        e = sbt::launch_batch_gang_reduce(B, n_gangs, st);
        if (e != hipSuccess) return fail(SBT_EDEVICE, "%s: gang reduce: %s", who, hipGetErrorString(e));
    }
    e = sbt::launch_batch_select(B, st);
    if (e != hipSuccess) return fail(SBT_EDEVICE, "%s: batch select: %s", who, hipGetErrorString(e));
    if (out->agent_trace)
        SBT_HIP(hipMemcpyAsync(out->agent_trace, B.etrace,
                               sizeof(double) * S.ev.size() * L.n_ckpt * p->agents,
                               hipMemcpyDeviceToDevice, st));
    return SBT_OK;
}

extern "C" int sbt_batch_run(const sbt_dev_batch *batch, sbt_mode mode, sbt_precision prec,
                             const sbt_solve_params *p, void *workspace, size_t workspace_bytes,
                             const sbt_dev_batch_result *out, void *stream) {
    return sbt_batch_run_tuned(batch, mode, prec, p, nullptr, workspace, workspace_bytes, out,
                               stream);
}

// ----------------------------------------------------------- host batch

namespace {

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

static int solve_batch_impl(const sbt_qubo *const *qs, int32_t E, const double *c0_scale,
                     int32_t same_start, sbt_mode mode, sbt_precision prec,
                     const sbt_solve_params *pp, sbt_batch_result *out, const char *who) {
    if (!qs || !out || !out->energy || !out->best_agent)
        return fail(SBT_EINVAL, "%s: NULL argument", who);
    if (E < 1) return fail(SBT_EINVAL, "%s: n_events must be >= 1", who);
    if (mode != SBT_BSB && mode != SBT_DSB && mode != SBT_ASB)
        return fail(SBT_EINVAL, "%s: unknown mode", who);
    if (prec != SBT_PREC_FP16 && prec != SBT_PREC_BF16)
        return fail(SBT_EUNSUPPORTED, "%s: batches hold 16-bit couplings (FP16 or BF16)", who);
    sbt_solve_params p;
    if (pp)
        p = *pp;
    else
        sbt_solve_params_default(&p);
    std::vector<int32_t> n(E);
    std::vector<int64_t> nnz(E);
    int64_t sum_n = 0, sum_nnz = 0;
    for (int32_t e = 0; e < E; ++e) {
        const sbt_qubo *q = qs[e];
        char what[32];
        snprintf(what, sizeof what, "event %d", e);
        const int vrc = sbt::validate_qubo_host(q, who, what, nullptr);
        if (vrc) return vrc;
        n[e] = q->n;
        nnz[e] = q->nnz;
        sum_n += q->n;
        sum_nnz += q->nnz;
    }
    std::vector<double> a(sum_n), b(std::max<int64_t>(sum_nnz, 1));
    std::vector<int32_t> rp(sum_n + E), col(std::max<int64_t>(sum_nnz, 1));
    {
        int64_t ro = 0, zo = 0;
        for (int32_t e = 0; e < E; ++e) {
            const sbt_qubo *q = qs[e];
            std::copy(q->a, q->a + q->n, a.begin() + ro);
            for (int32_t i = 0; i <= q->n; ++i) rp[ro + e + i] = static_cast<int32_t>(q->row_ptr[i]);
            std::copy(q->col, q->col + q->nnz, col.begin() + zo);
            std::copy(q->b, q->b + q->nnz, b.begin() + zo);
            ro += q->n;
            zo += q->nnz;
        }
    }
    int rc0 = check_batch_params(p, who);
    if (rc0) return rc0;
    // the tuned schedule for this batch's shape, if the tuning cache has one
    sbt_batch_tuning tu;
    rc0 = sbt_batch_tuning_lookup(n.data(), E, mode, prec, p.agents, &tu);
    if (rc0) return rc0;
    {
        Schedule S;
        rc0 = make_schedule(n.data(), nnz.data(), E, c0_scale, same_start, p, tu, S, who);
        if (rc0) return rc0;
    }
    const size_t ws_bytes = sbt_batch_workspace_bytes_tuned(n.data(), nnz.data(), E, &p, &tu);
    if (ws_bytes == 0) return SBT_EINVAL;
    const int n_ck = p.energy_every > 0 ? p.steps / p.energy_every : 0;
    if ((out->trace || out->agent_trace) && n_ck == 0)
        return fail(SBT_EINVAL, "%s: trace requested but energy_every gives no checkpoint", who);
    DevBuf da, drp, dcol, db, dws, dbe, dba, dbt, dae, dtr, dat;
    const size_t M = static_cast<size_t>(p.agents);
    if (hipMalloc(&da.p, sizeof(double) * sum_n) || hipMalloc(&drp.p, sizeof(int32_t) * rp.size()) ||
        hipMalloc(&dcol.p, sizeof(int32_t) * col.size()) || hipMalloc(&db.p, sizeof(double) * b.size()) ||
        hipMalloc(&dws.p, ws_bytes) || hipMalloc(&dbe.p, sizeof(double) * E) ||
        hipMalloc(&dba.p, sizeof(int32_t) * E) || hipMalloc(&dbt.p, sum_n) ||
        hipMalloc(&dae.p, sizeof(double) * E * M) ||
        (out->trace && hipMalloc(&dtr.p, sizeof(double) * E * n_ck)) ||
        (out->agent_trace && hipMalloc(&dat.p, sizeof(double) * E * n_ck * M)))
        return fail(SBT_ENOMEM, "%s: device allocation failed", who);
    hipStream_t st = nullptr;
    SBT_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() { (void)hipStreamDestroy(s); }
    } guard{st};
    SBT_HIP(hipMemcpyAsync(da.p, a.data(), sizeof(double) * sum_n, hipMemcpyHostToDevice, st));
    SBT_HIP(hipMemcpyAsync(drp.p, rp.data(), sizeof(int32_t) * rp.size(), hipMemcpyHostToDevice, st));
    SBT_HIP(hipMemcpyAsync(dcol.p, col.data(), sizeof(int32_t) * col.size(), hipMemcpyHostToDevice, st));
    SBT_HIP(hipMemcpyAsync(db.p, b.data(), sizeof(double) * b.size(), hipMemcpyHostToDevice, st));
    hipEvent_t e0, e1;
    SBT_HIP(hipEventCreate(&e0));
    SBT_HIP(hipEventCreate(&e1));
    struct EventGuard {
        hipEvent_t a, b;
        ~EventGuard() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } eg{e0, e1};
    SBT_HIP(hipEventRecord(e0, st));
    int rc = sbt_batch_plan_tuned(n.data(), nnz.data(), E, c0_scale, same_start, &p, &tu, dws.p,
                                  ws_bytes, st);
    if (rc < 0) return rc;
    sbt_dev_batch dbch{E, n.data(), nnz.data(), static_cast<const double *>(da.p),
                       static_cast<const int32_t *>(drp.p), static_cast<const int32_t *>(dcol.p),
                       static_cast<const double *>(db.p), nullptr};  // no target: full-length solves
    sbt_dev_batch_result dr{};
    dr.best_energy = static_cast<double *>(dbe.p);
    dr.best_agent = static_cast<int32_t *>(dba.p);
    dr.best_T = static_cast<int8_t *>(dbt.p);
    dr.agent_energy = static_cast<double *>(dae.p);
    dr.trace = static_cast<double *>(dtr.p);
    dr.agent_trace = static_cast<double *>(dat.p);
    rc = sbt_batch_run_tuned(&dbch, mode, prec, &p, &tu, dws.p, ws_bytes, &dr, st);
    if (rc) return rc;
    SBT_HIP(hipEventRecord(e1, st));
    SBT_HIP(hipMemcpyAsync(out->energy, dbe.p, sizeof(double) * E, hipMemcpyDeviceToHost, st));
    SBT_HIP(hipMemcpyAsync(out->best_agent, dba.p, sizeof(int32_t) * E, hipMemcpyDeviceToHost, st));
    if (out->T) SBT_HIP(hipMemcpyAsync(out->T, dbt.p, sum_n, hipMemcpyDeviceToHost, st));
    if (out->agent_energy)
        SBT_HIP(hipMemcpyAsync(out->agent_energy, dae.p, sizeof(double) * E * M, hipMemcpyDeviceToHost, st));
    if (out->trace)
        SBT_HIP(hipMemcpyAsync(out->trace, dtr.p, sizeof(double) * E * n_ck, hipMemcpyDeviceToHost, st));
    if (out->agent_trace)
        SBT_HIP(hipMemcpyAsync(out->agent_trace, dat.p, sizeof(double) * E * n_ck * M,
                               hipMemcpyDeviceToHost, st));
    SBT_HIP(hipStreamSynchronize(st));
    float ms = 0.0f;
    SBT_HIP(hipEventElapsedTime(&ms, e0, e1));
    out->elapsed_s = 1e-3 * ms;
    for (int32_t e = 0; e < E; ++e)
        if (std::isnan(out->energy[e]))
            return fail(SBT_EDEVICE, "%s: event %d: a gang of row bands timed out at a barrier", who, e);
    return SBT_OK;
}

extern "C" int sbt_wall_clock_hz(double *hz) {
    const char *who = "sbt_wall_clock_hz";
    sbt::clear_error();
    if (!hz) return fail(SBT_EINVAL, "%s: hz is NULL", who);
    int dev = 0, khz = 0;
    SBT_HIP(hipGetDevice(&dev));
    SBT_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    if (khz <= 0) return fail(SBT_EDEVICE, "%s: the device reports no wall clock rate", who);
    *hz = 1e3 * khz;
    return SBT_OK;
}

extern "C" int sbt_solve_batch(const sbt_qubo *const *qs, int32_t E, sbt_mode mode,
                               sbt_precision prec, const sbt_solve_params *p,
                               sbt_batch_result *out) {
    sbt::clear_error();
    return solve_batch_impl(qs, E, nullptr, 0, mode, prec, p, out, "sbt_solve_batch");
}

extern "C" int sbt_c0_scan(const sbt_qubo *q, sbt_mode mode, sbt_precision prec,
                           const sbt_solve_params *p, const double *factors, int32_t n_factors,
                           double *energy, int32_t *best_agent, int32_t *best_factor) {
    const char *who = "sbt_c0_scan";
    sbt::clear_error();
    if (!q || !factors || !energy || !best_agent || !best_factor)
        return fail(SBT_EINVAL, "%s: NULL argument", who);
    if (n_factors < 1) return fail(SBT_EINVAL, "%s: n_factors must be >= 1", who);
    std::vector<const sbt_qubo *> qs(static_cast<size_t>(n_factors), q);
    sbt_batch_result r{};
    r.energy = energy;
    r.best_agent = best_agent;
    const int rc = solve_batch_impl(qs.data(), n_factors, factors, 1, mode, prec, p, &r, who);
    if (rc) return rc;
    int32_t best = 0;
    for (int32_t k = 1; k < n_factors; ++k)
        if (energy[k] < energy[best]) best = k;
    *best_factor = best;
    return SBT_OK;
}
