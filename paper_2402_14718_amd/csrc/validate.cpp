// Host validation of a QUBO before it is uploaded (shared by sbt_solve,
// sbt_solve_batch and sbt_c0_scan).  Pure host code: no HIP calls.
//
// Eq. 13 needs b symmetric with a zero diagonal; the library stores both
// triangles in CSR with ascending columns.  The row pointers are checked
// completely before any row is walked, so a malformed row_ptr never
// indexes col or b out of range.
#include <algorithm>
#include <cmath>
#include <cstdint>

#include "common.hpp"

namespace sbt {

int validate_qubo_structure(const sbt_qubo *q, const char *who, const char *what) {
    if (!q) return fail(SBT_EINVAL, "%s: %s is NULL", who, what);
    if (q->n < 0 || q->nnz < 0) return fail(SBT_EINVAL, "%s: %s has a negative size", who, what);
    if (q->n == 0) return SBT_OK;
    if (!q->a || !q->row_ptr || (q->nnz > 0 && (!q->col || !q->b)))
        return fail(SBT_EINVAL, "%s: %s has a NULL array", who, what);
    if (q->row_ptr[0] != 0 || q->row_ptr[q->n] != q->nnz)
        return fail(SBT_EINVAL, "%s: %s row_ptr does not span [0, nnz]", who, what);
    for (int32_t i = 0; i < q->n; ++i)
        if (q->row_ptr[i + 1] < q->row_ptr[i])
            return fail(SBT_EINVAL, "%s: %s row_ptr decreases at row %d", who, what, i);
    for (int64_t e = 0; e < q->nnz; ++e)
        if (q->col[e] < 0 || q->col[e] >= q->n)
            return fail(SBT_EINVAL, "%s: %s column %d out of range", who, what, q->col[e]);
    return SBT_OK;
}

int validate_qubo_host(const sbt_qubo *q, const char *who, const char *what, int32_t *max_row) {
    if (!q) return fail(SBT_EINVAL, "%s: %s is NULL", who, what);
    if (q->n < 1) return fail(SBT_EINVAL, "%s: %s is empty (n = %d)", who, what, q->n);
    if (q->nnz < 0) return fail(SBT_EINVAL, "%s: %s has nnz < 0", who, what);
    if (!q->a || !q->row_ptr || (q->nnz > 0 && (!q->col || !q->b)))
        return fail(SBT_EINVAL, "%s: %s has a NULL array", who, what);
    if (q->row_ptr[0] != 0 || q->row_ptr[q->n] != q->nnz)
        return fail(SBT_EINVAL, "%s: %s row_ptr does not span [0, nnz]", who, what);
    // every row range inside [0, nnz] and non-decreasing, before any row is read
    int32_t mr = 0;
    for (int32_t i = 0; i < q->n; ++i) {
        const int64_t lo = q->row_ptr[i], hi = q->row_ptr[i + 1];
        if (lo < 0 || hi < lo || hi > q->nnz)
            return fail(SBT_EINVAL, "%s: %s row_ptr decreases or leaves [0, nnz] at row %d", who,
                        what, i);
        mr = static_cast<int32_t>(std::min<int64_t>(std::max<int64_t>(mr, hi - lo), INT32_MAX));
    }
    // columns in range, ascending, off the diagonal; values finite
    for (int32_t i = 0; i < q->n; ++i) {
        if (!std::isfinite(q->a[i])) return fail(SBT_EINVAL, "%s: %s a[%d] is not finite", who, what, i);
        const int64_t lo = q->row_ptr[i], hi = q->row_ptr[i + 1];
        for (int64_t e = lo; e < hi; ++e) {
            const int32_t j = q->col[e];
            if (j < 0 || j >= q->n)
                return fail(SBT_EINVAL, "%s: %s column %d out of range in row %d", who, what, j, i);
            if (j == i) return fail(SBT_EINVAL, "%s: %s diagonal entry in row %d", who, what, i);
            if (e > lo && q->col[e - 1] >= j)
                return fail(SBT_EINVAL, "%s: %s columns of row %d not ascending", who, what, i);
            if (!std::isfinite(q->b[e])) return fail(SBT_EINVAL, "%s: %s b is not finite", who, what);
        }
    }
    // symmetry, now that every row is known to be well formed
    for (int32_t i = 0; i < q->n; ++i) {
        for (int64_t e = q->row_ptr[i]; e < q->row_ptr[i + 1]; ++e) {
            const int32_t j = q->col[e];
            const int32_t *c0 = q->col + q->row_ptr[j];
            const int32_t *c1 = q->col + q->row_ptr[j + 1];
            const int32_t *f = std::lower_bound(c0, c1, i);
            if (f == c1 || *f != i || q->b[q->row_ptr[j] + (f - c0)] != q->b[e])
                return fail(SBT_EINVAL, "%s: %s b is not symmetric at (%d, %d)", who, what, i, j);
        }
    }
    if (max_row) *max_row = mr;
    return SBT_OK;
}

}  // namespace sbt
