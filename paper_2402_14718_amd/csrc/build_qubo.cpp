// Hits -> track QUBO (host, FP64).
//
// Paper sections "QUBO Formulation" (Eq. 13-15) and "QUBO Generation and
// Track Finding" (Eq. 16-17, the five-hit rule, pruning).  Readings where
// the paper is silent or garbled:
//   * doublets: hits on adjacent layers with |dphi| below the window,
//     decided by dot > 0 && |cross| < tan(window) * dot (no libm);
//   * curvature: signed transverse Menger curvature kappa = 1/R, mm^-1;
//   * delta-theta: angle between the (dr, dz) directions of the two
//     doublets, decided by a cross/dot test, valued with atan2;
//   * holes = last layer - first layer - 2 (always 0 for adjacent doublets);
//   * Eq. 15 with decaying exponentials: a = alpha (1 - e^{-|d0|/gamma}) +
//     beta (1 - e^{-|z0|/lambda}), a penalty in [0, alpha + beta);
//   * five-hit rule: an Eq.-17 quadruplet (i -> j) is kept if a passing
//     (j -> k) or (k -> i) exists; vacuous when fewer than five layers;
//   * b_ij: -S_ij for kept quadruplets, +1 for triplets sharing a hit that
//     are not shifted windows of one hit chain, otherwise 0.
// Every decision is a fixed-order IEEE expression (this file is compiled
// without floating-point contraction), so the enumeration is reproducible
// bit for bit by any implementation that evaluates the same expressions.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "common.hpp"
#include "sbtrack.h"

namespace {

constexpr double kTan0p1 = 0.10033467208545055;  // tan(0.1), FP64
constexpr double kPi = 3.14159265358979323846;

struct Hits {
    std::vector<int64_t> id;
    std::vector<int32_t> layer;
    std::vector<double> x, y, z;
};

struct Triplet {
    int32_t h[3];
    double kappa, dtheta, holes, d0, z0;
};

struct Quad {
    int32_t i, j;
    double s;
};

struct Coupling {
    int32_t u, v;  // u < v
    double w;
};

// Doublets between two layers: for each hit of the inner layer, scan the
// outer layer's hits whose azimuth lies in a slightly widened window (an
// atan2 pre-filter), then apply the exact cross/dot test.
void doublets_between(const Hits &H, const std::vector<int32_t> &inner,
                      const std::vector<int32_t> &outer, const sbt_build_params &p,
                      std::vector<std::pair<int32_t, int32_t>> &out) {
    if (inner.empty() || outer.empty()) return;
    std::vector<std::pair<double, int32_t>> ophi(outer.size());
    for (size_t k = 0; k < outer.size(); ++k) {
        int32_t h = outer[k];
        ophi[k] = {std::atan2(H.y[h], H.x[h]), h};
    }
    std::sort(ophi.begin(), ophi.end());
    const double win = std::atan(p.dphi_tan) + 1e-6;
    const bool all = !(win < 0.5 * kPi);
    auto accept = [&](int32_t a, int32_t b) {
        const double x1 = H.x[a], y1 = H.y[a], x2 = H.x[b], y2 = H.y[b];
        const double cross = x1 * y2 - y1 * x2;
        const double dot = x1 * x2 + y1 * y2;
        if (!(dot > 0.0 && std::fabs(cross) < p.dphi_tan * dot)) return;
        if (p.z0_max > 0.0) {
            const double r1 = std::sqrt(x1 * x1 + y1 * y1);
            const double r2 = std::sqrt(x2 * x2 + y2 * y2);
            const double z1 = H.z[a], z2 = H.z[b];
            const double z0 = z1 - r1 * (z2 - z1) / (r2 - r1);
            if (!(std::fabs(z0) <= p.z0_max)) return;
        }
        out.emplace_back(a, b);
    };
    auto scan = [&](int32_t a, double lo, double hi) {
        auto it = std::lower_bound(ophi.begin(), ophi.end(),
                                   std::make_pair(lo, INT32_MIN));
        for (; it != ophi.end() && it->first <= hi; ++it) accept(a, it->second);
    };
    for (int32_t a : inner) {
        if (all) {
            for (int32_t b : outer) accept(a, b);
            continue;
        }
        const double phi = std::atan2(H.y[a], H.x[a]);
        const double lo = phi - win, hi = phi + win;
        scan(a, std::max(lo, -kPi - 1.0), std::min(hi, kPi + 1.0));
        if (lo < -kPi) scan(a, lo + 2.0 * kPi, kPi + 1.0);
        if (hi > kPi) scan(a, -kPi - 1.0, hi - 2.0 * kPi);
    }
}

// Triplet geometry in the canonical evaluation order.
bool make_triplet(const Hits &H, int32_t a, int32_t b, int32_t c,
                  const sbt_build_params &p, Triplet &t) {
    const double x1 = H.x[a], y1 = H.y[a], z1 = H.z[a];
    const double x2 = H.x[b], y2 = H.y[b], z2 = H.z[b];
    const double x3 = H.x[c], y3 = H.y[c], z3 = H.z[c];
    const double ux = x2 - x1, uy = y2 - y1;
    const double vx = x3 - x2, vy = y3 - y2;
    const double wx = x3 - x1, wy = y3 - y1;
    const double cr = ux * vy - uy * vx;
    const double nu = std::sqrt(ux * ux + uy * uy);
    const double nv = std::sqrt(vx * vx + vy * vy);
    const double nw = std::sqrt(wx * wx + wy * wy);
    const double kappa = (2.0 * cr) / ((nu * nv) * nw);
    const double r1 = std::sqrt(x1 * x1 + y1 * y1);
    const double r2 = std::sqrt(x2 * x2 + y2 * y2);
    const double r3 = std::sqrt(x3 * x3 + y3 * y3);
    const double d1r = r2 - r1, d1z = z2 - z1;
    const double d2r = r3 - r2, d2z = z3 - z2;
    const double tcross = d1r * d2z - d1z * d2r;
    const double tdot = d1r * d2r + d1z * d2z;
    const int holes = H.layer[c] - H.layer[a] - 2;
    if (holes > p.max_holes) return false;
    if (!(std::fabs(kappa) <= p.curv_max)) return false;
    if (!(tdot > 0.0 && std::fabs(tcross) <= p.dtheta_tan * tdot)) return false;
    // transverse impact parameter: circle through the hits, centre relative
    // to the first hit
    const double bb = ux * ux + uy * uy;
    const double cc = wx * wx + wy * wy;
    const double den = 2.0 * (ux * wy - uy * wx);
    double d0;
    if (den != 0.0) {
        const double ocx = (wy * bb - uy * cc) / den;
        const double ocy = (ux * cc - wx * bb) / den;
        const double xc = x1 + ocx, yc = y1 + ocy;
        const double rad = std::sqrt(ocx * ocx + ocy * ocy);
        d0 = std::fabs(std::sqrt(xc * xc + yc * yc) - rad);
    } else {
        d0 = std::fabs(x1 * wy - y1 * wx) / nw;
    }
    t.h[0] = a;
    t.h[1] = b;
    t.h[2] = c;
    t.kappa = kappa;
    t.dtheta = std::atan2(std::fabs(tcross), tdot);
    t.holes = static_cast<double>(holes);
    t.d0 = d0;
    t.z0 = z1 - r1 * d1z / d1r;
    return true;
}

enum class Relation { None, Shift1, Shift2, Conflict };

Relation relate(const int32_t *p, const int32_t *q) {
    bool share = false;
    for (int s = 0; s < 3; ++s)
        for (int u = 0; u < 3; ++u) share |= (p[s] == q[u]);
    if (!share) return Relation::None;
    if ((p[1] == q[0] && p[2] == q[1]) || (q[1] == p[0] && q[2] == p[1])) return Relation::Shift1;
    if (p[2] == q[0] || q[2] == p[0]) return Relation::Shift2;
    return Relation::Conflict;
}

template <class T>
T *dup_array(const std::vector<T> &v) {
    T *p = static_cast<T *>(std::malloc(std::max<size_t>(1, v.size()) * sizeof(T)));
    if (!p) throw std::bad_alloc();
    if (!v.empty()) std::memcpy(p, v.data(), v.size() * sizeof(T));
    return p;
}

int build_impl(const sbt_hit *hits, int64_t n_hits, const sbt_build_params &p, sbt_qubo **out) {
    // hits ordered by id: internal index order == canonical id order
    std::vector<int64_t> order(static_cast<size_t>(n_hits));
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(),
              [&](int64_t u, int64_t v) { return hits[u].hit_id < hits[v].hit_id; });
    Hits H;
    H.id.resize(n_hits);
    H.layer.resize(n_hits);
    H.x.resize(n_hits);
    H.y.resize(n_hits);
    H.z.resize(n_hits);
    int32_t n_layers = 0;
    for (int64_t k = 0; k < n_hits; ++k) {
        const sbt_hit &h = hits[order[k]];
        if (k > 0 && h.hit_id == H.id[k - 1])
            return sbt::fail(SBT_EINVAL, "sbt_build_qubo: duplicate hit id %lld",
                             static_cast<long long>(h.hit_id));
        H.id[k] = h.hit_id;
        H.layer[k] = h.layer;
        H.x[k] = h.x;
        H.y[k] = h.y;
        H.z[k] = h.z;
        n_layers = std::max(n_layers, h.layer + 1);
    }
    int32_t mth = p.min_track_hits >= 0 ? p.min_track_hits : std::min(5, n_layers);
    if (mth > 5)
        return sbt::fail(SBT_EUNSUPPORTED, "sbt_build_qubo: min_track_hits > 5 not implemented");

    std::vector<std::vector<int32_t>> by_layer(n_layers);
    for (int32_t k = 0; k < static_cast<int32_t>(n_hits); ++k) by_layer[H.layer[k]].push_back(k);

    // 1. doublets, sorted by (inner id, outer id)
    std::vector<std::pair<int32_t, int32_t>> dbl;
    for (int32_t L = 0; L + 1 < n_layers; ++L) doublets_between(H, by_layer[L], by_layer[L + 1], p, dbl);
    std::sort(dbl.begin(), dbl.end());

    // outgoing adjacency (CSR over hits, targets ascending)
    std::vector<int32_t> out_ptr(n_hits + 1, 0), out_dst(dbl.size());
    for (auto &d : dbl) out_ptr[d.first + 1]++;
    for (int64_t k = 0; k < n_hits; ++k) out_ptr[k + 1] += out_ptr[k];
    {
        std::vector<int32_t> fill(out_ptr.begin(), out_ptr.end() - 1);
        for (auto &d : dbl) out_dst[fill[d.first]++] = d.second;
    }

    // 2. triplets (Eq. 16), produced in (h1, h2, h3) order
    std::vector<Triplet> trips;
    for (auto &d : dbl) {
        for (int32_t e = out_ptr[d.second]; e < out_ptr[d.second + 1]; ++e) {
            Triplet t;
            if (make_triplet(H, d.first, d.second, out_dst[e], p, t)) trips.push_back(t);
        }
    }

    // 3. quadruplets (Eq. 14, 17): i = (h1,h2,h3) -> j = (h2,h3,h4)
    auto first_pair_less = [](const Triplet &t, std::pair<int32_t, int32_t> k) {
        return t.h[0] < k.first || (t.h[0] == k.first && t.h[1] < k.second);
    };
    std::vector<Quad> quads;
    for (int32_t i = 0; i < static_cast<int32_t>(trips.size()); ++i) {
        const Triplet &ti = trips[i];
        std::pair<int32_t, int32_t> key{ti.h[1], ti.h[2]};
        auto it = std::lower_bound(trips.begin(), trips.end(), key, first_pair_less);
        for (; it != trips.end() && it->h[0] == key.first && it->h[1] == key.second; ++it) {
            const double dk = std::fabs(ti.kappa - it->kappa);
            if (!(dk <= p.dcurv_max)) continue;
            const double hsum = 1.0 + ti.holes + it->holes;
            const double s = (1.0 - 0.5 * (dk + std::max(ti.dtheta, it->dtheta))) / (hsum * hsum);
            if (!(s > p.s_min)) continue;
            quads.push_back({i, static_cast<int32_t>(it - trips.begin()), s});
        }
    }

    // 4. five-hit rule, one pass over the passing set
    std::vector<Quad> kept;
    if (mth >= 5) {
        std::vector<char> has_out(trips.size(), 0), has_in(trips.size(), 0);
        for (auto &q : quads) {
            has_out[q.i] = 1;
            has_in[q.j] = 1;
        }
        for (auto &q : quads)
            if (has_out[q.j] || has_in[q.i]) kept.push_back(q);
    } else {
        kept = quads;
    }

    // 5. triplets in a kept quadruplet survive; canonical ids in order
    std::vector<int32_t> new_id(trips.size(), -1);
    for (auto &q : kept) new_id[q.i] = new_id[q.j] = 0;
    int32_t n = 0;
    for (auto &v : new_id)
        if (v == 0) v = n++;
    std::vector<int32_t> alive(n);
    for (int32_t t = 0; t < static_cast<int32_t>(trips.size()); ++t)
        if (new_id[t] >= 0) alive[new_id[t]] = t;

    // 6. bias weights (Eq. 15)
    std::vector<double> a(n);
    std::vector<int64_t> trip_ids(3 * static_cast<size_t>(n));
    for (int32_t k = 0; k < n; ++k) {
        const Triplet &t = trips[alive[k]];
        a[k] = p.alpha * (1.0 - std::exp(-std::fabs(t.d0) / p.gamma_)) +
               p.beta * (1.0 - std::exp(-std::fabs(t.z0) / p.lambda_));
        for (int s = 0; s < 3; ++s) trip_ids[3 * k + s] = H.id[t.h[s]];
    }

    // 7. couplings (Eq. 13): rewards of kept quadruplets, conflicts via
    //    the triplets that contain each hit
    std::vector<Coupling> cpl;
    for (auto &q : kept) {
        int32_t u = new_id[q.i], v = new_id[q.j];
        cpl.push_back({std::min(u, v), std::max(u, v), -q.s});
    }
    {
        std::vector<std::pair<int32_t, int32_t>> memb;  // (hit, triplet)
        memb.reserve(3 * static_cast<size_t>(n));
        for (int32_t k = 0; k < n; ++k)
            for (int s = 0; s < 3; ++s) memb.emplace_back(trips[alive[k]].h[s], k);
        std::sort(memb.begin(), memb.end());
        std::vector<Coupling> conf;
        for (size_t lo = 0; lo < memb.size();) {
            size_t hi = lo;
            while (hi < memb.size() && memb[hi].first == memb[lo].first) ++hi;
            for (size_t u = lo; u < hi; ++u)
                for (size_t v = u + 1; v < hi; ++v) {
                    int32_t tu = memb[u].second, tv = memb[v].second;
                    if (relate(trips[alive[tu]].h, trips[alive[tv]].h) == Relation::Conflict)
                        conf.push_back({std::min(tu, tv), std::max(tu, tv), 1.0});
                }
            lo = hi;
        }
        std::sort(conf.begin(), conf.end(), [](const Coupling &l, const Coupling &r) {
            return l.u < r.u || (l.u == r.u && l.v < r.v);
        });
        for (size_t k = 0; k < conf.size(); ++k)
            if (k == 0 || conf[k].u != conf[k - 1].u || conf[k].v != conf[k - 1].v)
                cpl.push_back(conf[k]);
    }

    // symmetric CSR, ascending columns
    std::vector<int64_t> row_ptr(n + 1, 0);
    for (auto &c : cpl) {
        row_ptr[c.u + 1]++;
        row_ptr[c.v + 1]++;
    }
    for (int32_t k = 0; k < n; ++k) row_ptr[k + 1] += row_ptr[k];
    const int64_t nnz = row_ptr[n];
    std::vector<std::pair<int32_t, double>> ent(nnz);
    {
        std::vector<int64_t> fill(row_ptr.begin(), row_ptr.end() - 1);
        for (auto &c : cpl) {
            ent[fill[c.u]++] = {c.v, c.w};
            ent[fill[c.v]++] = {c.u, c.w};
        }
    }
    std::vector<int32_t> col(nnz);
    std::vector<double> bv(nnz);
    for (int32_t k = 0; k < n; ++k) {
        std::sort(ent.begin() + row_ptr[k], ent.begin() + row_ptr[k + 1],
                  [](const std::pair<int32_t, double> &l, const std::pair<int32_t, double> &r) {
                      return l.first < r.first;
                  });
        for (int64_t e = row_ptr[k]; e < row_ptr[k + 1]; ++e) {
            col[e] = ent[e].first;
            bv[e] = ent[e].second;
        }
    }

    sbt_qubo *q = static_cast<sbt_qubo *>(std::calloc(1, sizeof(sbt_qubo)));
    if (!q) throw std::bad_alloc();
    q->n = n;
    q->nnz = nnz;
    try {
        q->a = dup_array(a);
        q->row_ptr = dup_array(row_ptr);
        q->col = dup_array(col);
        q->b = dup_array(bv);
        q->trip_hits = dup_array(trip_ids);
    } catch (...) {
        sbt_qubo_free(q);
        throw;
    }
    *out = q;
    return SBT_OK;
}

}  // namespace

extern "C" void sbt_build_params_default(sbt_build_params *p) {
    if (!p) return;
    p->dphi_tan = kTan0p1;
    p->z0_max = 0.0;
    p->curv_max = 8e-4;
    p->dtheta_tan = kTan0p1;
    p->dcurv_max = 1e-4;
    p->s_min = 0.2;
    p->max_holes = 1;
    p->min_track_hits = -1;
    p->alpha = 0.5;
    p->beta = 0.2;
    p->gamma_ = 1.0;
    p->lambda_ = 0.5;
}

int sbt::check_build_inputs(const sbt_hit *hits, int64_t n_hits, const sbt_build_params *pp,
                            sbt_qubo **out, sbt_build_params *p, const char *who) {
    if (!out) return sbt::fail(SBT_EINVAL, "%s: out is NULL", who);
    *out = nullptr;
    if (n_hits < 0 || n_hits > INT32_MAX / 2)
        return sbt::fail(SBT_EINVAL, "%s: n_hits %lld out of range", who,
                         static_cast<long long>(n_hits));
    if (n_hits > 0 && !hits) return sbt::fail(SBT_EINVAL, "%s: hits is NULL", who);
    if (pp)
        *p = *pp;
    else
        sbt_build_params_default(p);
    if (!(p->dphi_tan > 0.0) || !(p->dtheta_tan > 0.0) || !(p->gamma_ > 0.0) ||
        !(p->lambda_ > 0.0) || !std::isfinite(p->curv_max) || !std::isfinite(p->dcurv_max) ||
        !std::isfinite(p->s_min))
        return sbt::fail(SBT_EINVAL, "%s: invalid parameters", who);
    for (int64_t k = 0; k < n_hits; ++k) {
        const sbt_hit &h = hits[k];
        if (!std::isfinite(h.x) || !std::isfinite(h.y) || !std::isfinite(h.z))
            return sbt::fail(SBT_EINVAL, "%s: hit %lld has a non-finite coordinate", who,
                             static_cast<long long>(k));
        if (h.layer < 0 || h.layer > 4096)
            return sbt::fail(SBT_EINVAL, "%s: hit %lld has layer %d", who,
                             static_cast<long long>(k), h.layer);
    }
    return SBT_OK;
}

extern "C" int sbt_build_qubo(const sbt_hit *hits, int64_t n_hits, const sbt_build_params *pp,
                              sbt_qubo **out) {
    sbt::clear_error();
    sbt_build_params p;
    const int rc = sbt::check_build_inputs(hits, n_hits, pp, out, &p, "sbt_build_qubo");
    if (rc) return rc;
    try {
        return build_impl(hits, n_hits, p, out);
    } catch (const std::bad_alloc &) {
        return sbt::fail(SBT_ENOMEM, "sbt_build_qubo: out of host memory");
    }
}

extern "C" void sbt_qubo_free(sbt_qubo *q) {
    if (!q) return;
    std::free(q->a);
    std::free(q->row_ptr);
    std::free(q->col);
    std::free(q->b);
    std::free(q->trip_hits);
    std::free(q);
}

extern "C" int sbt_energy(const sbt_qubo *q, const int8_t *T, double *energy) {
    sbt::clear_error();
    if (!q || !T || !energy) return sbt::fail(SBT_EINVAL, "sbt_energy: NULL argument");
    const int vrc = sbt::validate_qubo_structure(q, "sbt_energy", "qubo");
    if (vrc) return vrc;
    // Neumaier-compensated sum of a_i T_i and b_ij T_i T_j over j > i
    double s = 0.0, c = 0.0;
    auto add = [&](double v) {
        const double t = s + v;
        if (std::fabs(s) >= std::fabs(v))
            c += (s - t) + v;
        else
            c += (v - t) + s;
        s = t;
    };
    for (int32_t i = 0; i < q->n; ++i) {
        if (T[i] != 0 && T[i] != 1) return sbt::fail(SBT_EINVAL, "sbt_energy: T[%d] not 0/1", i);
        const double ti = T[i];
        add(q->a[i] * ti);
        for (int64_t e = q->row_ptr[i]; e < q->row_ptr[i + 1]; ++e) {
            const int32_t j = q->col[e];
            if (j > i) add(q->b[e] * (ti * static_cast<double>(T[j])));
        }
    }
    *energy = s + c;
    return SBT_OK;
}
