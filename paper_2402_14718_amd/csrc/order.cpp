// Spin orderings of a triplet QUBO (host).
//
// The streaming SB kernel gathers x_j for every coupling of row i; its
// caches work best when coupled triplets sit at nearby indices.  Triplets
// that share hits lie along one track, so they have nearly the same
// azimuth: sorting triplets by the azimuth of their middle hit (then its z)
// puts the non-zeros of b near the diagonal.  The order changes nothing in
// the problem: O(P T) on the permuted QUBO equals O(T) on the original.
//
// The azimuth is compared through an exact monotone stand-in ("diamond
// angle", one division, no transcendental): for d = |x| + |y| > 0,
//   key = 1 - x/d  (y >= 0),   key = 3 + x/d  (y < 0),
// which rises from 0 at phi = 0 through 1, 2, 3 at pi/2, pi, 3pi/2 to 4.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <new>
#include <utility>
#include <vector>

#include "common.hpp"
#include "sbtrack.h"

namespace {

double diamond_angle(double x, double y) {
    const double d = std::fabs(x) + std::fabs(y);
    if (d == 0.0) return 0.0;
    const double t = x / d;
    return y >= 0.0 ? 1.0 - t : 3.0 + t;
}

template <class T>
T *alloc_array(size_t n) {
    T *p = static_cast<T *>(std::malloc(std::max<size_t>(1, n) * sizeof(T)));
    if (!p) throw std::bad_alloc();
    return p;
}

int phi_order_impl(const sbt_qubo *q, const sbt_hit *hits, int64_t n_hits, int32_t *perm) {
    std::vector<int64_t> by_id(static_cast<size_t>(n_hits));
    std::iota(by_id.begin(), by_id.end(), 0);
    std::sort(by_id.begin(), by_id.end(),
              [&](int64_t u, int64_t v) { return hits[u].hit_id < hits[v].hit_id; });
    const int32_t n = q->n;
    std::vector<double> key(n), zk(n);
    for (int32_t i = 0; i < n; ++i) {
        const int64_t id = q->trip_hits[3 * static_cast<int64_t>(i) + 1];
        auto it = std::lower_bound(by_id.begin(), by_id.end(), id,
                                   [&](int64_t u, int64_t v) { return hits[u].hit_id < v; });
        if (it == by_id.end() || hits[*it].hit_id != id)
            return sbt::fail(SBT_EINVAL, "sbt_phi_order: triplet %d names hit id %lld, not given",
                             i, static_cast<long long>(id));
        const sbt_hit &h = hits[*it];
        key[i] = diamond_angle(h.x, h.y);
        zk[i] = h.z;
    }
    std::vector<int32_t> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int32_t u, int32_t v) {
        if (key[u] != key[v]) return key[u] < key[v];
        if (zk[u] != zk[v]) return zk[u] < zk[v];
        return u < v;
    });
    std::memcpy(perm, idx.data(), sizeof(int32_t) * static_cast<size_t>(n));
    return SBT_OK;
}

int permute_impl(const sbt_qubo *q, const int32_t *perm, sbt_qubo **out) {
    const int32_t n = q->n;
    std::vector<int32_t> inv(n, -1);
    for (int32_t k = 0; k < n; ++k) {
        const int32_t o = perm[k];
        if (o < 0 || o >= n || inv[o] >= 0)
            return sbt::fail(SBT_EINVAL, "sbt_qubo_permute: perm is not a permutation of 0..%d",
                             n - 1);
        inv[o] = k;
    }
    sbt_qubo *r = static_cast<sbt_qubo *>(std::calloc(1, sizeof(sbt_qubo)));
    if (!r) throw std::bad_alloc();
    r->n = n;
    r->nnz = q->nnz;
    try {
        r->a = alloc_array<double>(n);
        r->row_ptr = alloc_array<int64_t>(static_cast<size_t>(n) + 1);
        r->col = alloc_array<int32_t>(static_cast<size_t>(q->nnz));
        r->b = alloc_array<double>(static_cast<size_t>(q->nnz));
        r->trip_hits = alloc_array<int64_t>(3 * static_cast<size_t>(n));
    } catch (...) {
        sbt_qubo_free(r);
        throw;
    }
    std::vector<std::pair<int32_t, double>> row;
    int64_t e = 0;
    r->row_ptr[0] = 0;
    for (int32_t k = 0; k < n; ++k) {
        const int32_t o = perm[k];
        r->a[k] = q->a[o];
        for (int c = 0; c < 3; ++c) r->trip_hits[3 * static_cast<int64_t>(k) + c] =
            q->trip_hits[3 * static_cast<int64_t>(o) + c];
        row.clear();
        for (int64_t p = q->row_ptr[o]; p < q->row_ptr[o + 1]; ++p)
            row.emplace_back(inv[q->col[p]], q->b[p]);
        std::sort(row.begin(), row.end(),
                  [](const std::pair<int32_t, double> &u, const std::pair<int32_t, double> &v) {
                      return u.first < v.first;
                  });
        for (const auto &cv : row) {
            r->col[e] = cv.first;
            r->b[e] = cv.second;
            ++e;
        }
        r->row_ptr[k + 1] = e;
    }
    *out = r;
    return SBT_OK;
}

int check_qubo_shape(const sbt_qubo *q, const char *who) {
    if (!q) return sbt::fail(SBT_EINVAL, "%s: QUBO is NULL", who);
    if (q->n < 0 || q->nnz < 0) return sbt::fail(SBT_EINVAL, "%s: negative size", who);
    if (q->n > 0 && (!q->a || !q->row_ptr || !q->trip_hits))
        return sbt::fail(SBT_EINVAL, "%s: QUBO array is NULL", who);
    if (q->nnz > 0 && (!q->col || !q->b)) return sbt::fail(SBT_EINVAL, "%s: QUBO array is NULL", who);
    if (q->n > 0 && (q->row_ptr[0] != 0 || q->row_ptr[q->n] != q->nnz))
        return sbt::fail(SBT_EINVAL, "%s: row_ptr does not span nnz", who);
    for (int32_t i = 0; i < q->n; ++i)
        if (q->row_ptr[i + 1] < q->row_ptr[i])
            return sbt::fail(SBT_EINVAL, "%s: row_ptr decreases at row %d", who, i);
    for (int64_t p = 0; p < q->nnz; ++p)
        if (q->col[p] < 0 || q->col[p] >= q->n)
            return sbt::fail(SBT_EINVAL, "%s: column %d out of range", who, q->col[p]);
    return SBT_OK;
}

}  // namespace

extern "C" int sbt_phi_order(const sbt_qubo *q, const sbt_hit *hits, int64_t n_hits,
                             int32_t *perm) {
    sbt::clear_error();
    int rc = check_qubo_shape(q, "sbt_phi_order");
    if (rc) return rc;
    if (n_hits < 0 || (n_hits > 0 && !hits) || (q->n > 0 && !perm))
        return sbt::fail(SBT_EINVAL, "sbt_phi_order: invalid hits or perm");
    try {
        return phi_order_impl(q, hits, n_hits, perm);
    } catch (const std::bad_alloc &) {
        return sbt::fail(SBT_ENOMEM, "sbt_phi_order: out of host memory");
    }
}

extern "C" int sbt_qubo_permute(const sbt_qubo *q, const int32_t *perm, sbt_qubo **out) {
    sbt::clear_error();
    if (!out) return sbt::fail(SBT_EINVAL, "sbt_qubo_permute: out is NULL");
    *out = nullptr;
    int rc = check_qubo_shape(q, "sbt_qubo_permute");
    if (rc) return rc;
    if (q->n > 0 && !perm) return sbt::fail(SBT_EINVAL, "sbt_qubo_permute: perm is NULL");
    try {
        return permute_impl(q, perm, out);
    } catch (const std::bad_alloc &) {
        return sbt::fail(SBT_ENOMEM, "sbt_qubo_permute: out of host memory");
    }
}
