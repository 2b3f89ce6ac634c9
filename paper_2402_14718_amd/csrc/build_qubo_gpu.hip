// Hits -> track QUBO on the GPU (FP64).
//
// The construction of sbt_build_qubo (sections "QUBO Formulation", Eq.
// 13-15, and "QUBO Generation and Track Finding", Eq. 16-17 and the
// five-hit rule) with the same readings and the same fixed-order IEEE
// expressions (this file is compiled without floating-point contraction),
// so the enumeration -- doublets, triplets, quadruplets, conflicts, the
// triplet order and the CSR structure -- is the host builder's.  Values
// that pass through exp (the Eq. 15 biases) or atan2 (the delta-theta term
// of Eq. 14) come from the device math library and can differ from the
// host's in the last place.
//
// The host sorts the hits by id and lists each layer's hits by azimuth
// (O(n log n) on the hits).  Every combinatorial stage runs on the device
// as count -> exclusive scan -> fill passes, with device radix sorts where
// the host sorts:
//   doublets      one thread per inner hit: binary search of the outer
//                 layer's azimuth window, exact cross/dot test;
//   triplets      one thread per doublet, over the middle hit's outgoing
//                 doublets (produced in (h1, h2, h3) order);
//   quadruplets   one thread per triplet, over the triplets that start with
//                 its last two hits (binary search);
//   five-hit rule, surviving triplets (scan = new index), Eq. 15 biases;
//   conflicts     one thread per (hit, triplet) membership, over the other
//                 triplets holding that hit, then sort + unique;
//   CSR           row counts, scan, scattered fill, one thread per row
//                 sorting its columns.
#include <hip/hip_runtime.h>

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <utility>
#include <vector>

#include "common.hpp"
#include "sbtrack.h"

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kTPB = 256;

struct GTrip {
    int32_t h0, h1, h2, holes;
    double kappa, dtheta, d0, z0;
};

struct Geo {
    const double *x, *y, *z, *phi;  // hits in id order; phi = host atan2
    const int32_t *layer;
};

struct Cuts {
    double dphi_tan, z0_max, curv_max, dtheta_tan, dcurv_max, s_min;
    double alpha, beta, gamma_, lambda_;
    double win;  // azimuth pre-filter half-width
    int32_t all;  // window covers every outer hit
    int32_t max_holes;
};

unsigned blocks(int64_t n) { return static_cast<unsigned>((n + kTPB - 1) / kTPB); }

template <class T>
struct DArr {
    T *p = nullptr;
    DArr() = default;
    DArr(const DArr &) = delete;
    DArr &operator=(const DArr &) = delete;
    ~DArr() {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(int64_t n) {
        if (p) (void)hipFree(p);
        p = nullptr;
        return hipMalloc(reinterpret_cast<void **>(&p), sizeof(T) * static_cast<size_t>(std::max<int64_t>(n, 1)));
    }
};

// ------------------------------------------------------------- doublets

__device__ __forceinline__ bool accept_doublet(const Geo &G, const Cuts &C, int32_t a, int32_t b) {
    const double x1 = G.x[a], y1 = G.y[a], x2 = G.x[b], y2 = G.y[b];
    const double cross = x1 * y2 - y1 * x2;
    const double dot = x1 * x2 + y1 * y2;
    if (!(dot > 0.0 && fabs(cross) < C.dphi_tan * dot)) return false;
    if (C.z0_max > 0.0) {
        const double r1 = sqrt(x1 * x1 + y1 * y1);
        const double r2 = sqrt(x2 * x2 + y2 * y2);
        const double z1 = G.z[a], z2 = G.z[b];
        const double z0 = z1 - r1 * (z2 - z1) / (r2 - r1);
        if (!(fabs(z0) <= C.z0_max)) return false;
    }
    return true;
}

// FILL = false: cnt[k] = doublets of inner hit k; FILL = true: write keys
// (inner << 32 | outer) at off[k].
template <bool FILL>
__global__ void doublets_kernel(int64_t n_inner, const int32_t *__restrict__ inner, Geo G, Cuts C,
                                const int32_t *__restrict__ lay_off,
                                const int32_t *__restrict__ phi_idx,
                                const double *__restrict__ phi_val, int64_t *__restrict__ cnt,
                                const int64_t *__restrict__ off, uint64_t *__restrict__ keys) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kTPB + threadIdx.x;
    if (k >= n_inner) return;
    const int32_t a = inner[k];
    const int32_t L = G.layer[a];
    const int32_t s = lay_off[L + 1], e = lay_off[L + 2];
    int64_t c = 0;
    int64_t at = FILL ? off[k] : 0;
    auto take = [&](int32_t b) {
        if (!accept_doublet(G, C, a, b)) return;
        if (FILL) keys[at++] = (static_cast<uint64_t>(a) << 32) | static_cast<uint32_t>(b);
        ++c;
    };
    auto scan = [&](double lo, double hi) {
        int32_t l = s, r = e;  // first position with phi >= lo
        while (l < r) {
            const int32_t m = l + (r - l) / 2;
            if (phi_val[m] < lo)
                l = m + 1;
            else
                r = m;
        }
        for (int32_t q = l; q < e && phi_val[q] <= hi; ++q) take(phi_idx[q]);
    };
    if (C.all) {
        for (int32_t q = s; q < e; ++q) take(phi_idx[q]);
    } else {
        const double phi = G.phi[a];
        const double lo = phi - C.win, hi = phi + C.win;
        scan(fmax(lo, -kPi - 1.0), fmin(hi, kPi + 1.0));
        if (lo < -kPi) scan(lo + 2.0 * kPi, kPi + 1.0);
        if (hi > kPi) scan(-kPi - 1.0, hi - 2.0 * kPi);
    }
    if (!FILL) cnt[k] = c;
}

__global__ void decode_pairs(int64_t n, const uint64_t *__restrict__ keys, int32_t *__restrict__ hi,
                             int32_t *__restrict__ lo) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kTPB + threadIdx.x;
    if (k >= n) return;
    hi[k] = static_cast<int32_t>(keys[k] >> 32);
    lo[k] = static_cast<int32_t>(keys[k] & 0xFFFFFFFFu);
}

__global__ void count_first(int64_t n, const int32_t *__restrict__ first, int64_t *__restrict__ cnt) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kTPB + threadIdx.x;
    if (k >= n) return;
    atomicAdd(reinterpret_cast<unsigned long long *>(cnt + first[k]), 1ull);
}

// ------------------------------------------------------------- triplets

__device__ bool make_triplet(const Geo &G, const Cuts &C, int32_t a, int32_t b, int32_t c,
                             GTrip &t) {
    const double x1 = G.x[a], y1 = G.y[a], z1 = G.z[a];
    const double x2 = G.x[b], y2 = G.y[b], z2 = G.z[b];
    const double x3 = G.x[c], y3 = G.y[c], z3 = G.z[c];
    const double ux = x2 - x1, uy = y2 - y1;
    const double vx = x3 - x2, vy = y3 - y2;
    const double wx = x3 - x1, wy = y3 - y1;
    const double cr = ux * vy - uy * vx;
    const double nu = sqrt(ux * ux + uy * uy);
    const double nv = sqrt(vx * vx + vy * vy);
    const double nw = sqrt(wx * wx + wy * wy);
    const double kappa = (2.0 * cr) / ((nu * nv) * nw);
    const double r1 = sqrt(x1 * x1 + y1 * y1);
    const double r2 = sqrt(x2 * x2 + y2 * y2);
    const double r3 = sqrt(x3 * x3 + y3 * y3);
    const double d1r = r2 - r1, d1z = z2 - z1;
    const double d2r = r3 - r2, d2z = z3 - z2;
    const double tcross = d1r * d2z - d1z * d2r;
    const double tdot = d1r * d2r + d1z * d2z;
    const int holes = G.layer[c] - G.layer[a] - 2;
    if (holes > C.max_holes) return false;
    if (!(fabs(kappa) <= C.curv_max)) return false;
    if (!(tdot > 0.0 && fabs(tcross) <= C.dtheta_tan * tdot)) return false;
    const double bb = ux * ux + uy * uy;
    const double cc = wx * wx + wy * wy;
    const double den = 2.0 * (ux * wy - uy * wx);
    double d0;
    if (den != 0.0) {
        const double ocx = (wy * bb - uy * cc) / den;
        const double ocy = (ux * cc - wx * bb) / den;
        const double xc = x1 + ocx, yc = y1 + ocy;
        const double rad = sqrt(ocx * ocx + ocy * ocy);
        d0 = fabs(sqrt(xc * xc + yc * yc) - rad);
    } else {
        d0 = fabs(x1 * wy - y1 * wx) / nw;
    }
    t.h0 = a;
    t.h1 = b;
    t.h2 = c;
    t.holes = holes;
    t.kappa = kappa;
    t.dtheta = atan2(fabs(tcross), tdot);
    t.d0 = d0;
    t.z0 = z1 - r1 * d1z / d1r;
    return true;
}

template <bool FILL>
__global__ void triplets_kernel(int64_t n_dbl, const int32_t *__restrict__ din,
                                const int32_t *__restrict__ dout,
                                const int64_t *__restrict__ out_ptr, Geo G, Cuts C,
                                int64_t *__restrict__ cnt, const int64_t *__restrict__ off,
                                GTrip *__restrict__ trips) {
    const int64_t d = static_cast<int64_t>(blockIdx.x) * kTPB + threadIdx.x;
    if (d >= n_dbl) return;
    const int32_t a = din[d], b = dout[d];
    int64_t c = 0;
    int64_t at = FILL ? off[d] : 0;
    for (int64_t e = out_ptr[b]; e < out_ptr[b + 1]; ++e) {
        GTrip t;
        if (!make_triplet(G, C, a, b, dout[e], t)) continue;
        if (FILL) trips[at++] = t;
        ++c;
    }
    if (!FILL) cnt[d] = c;
}

// ---------------------------------------------------------- quadruplets

template <bool FILL>
__global__ void quads_kernel(int64_t n_trip, const GTrip *__restrict__ T, Cuts C,
                             int64_t *__restrict__ cnt, const int64_t *__restrict__ off,
                             int32_t *__restrict__ qi, int32_t *__restrict__ qj,
                             double *__restrict__ qs) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kTPB + threadIdx.x;
    if (i >= n_trip) return;
    const GTrip ti = T[i];
    // first triplet with (h0, h1) >= (ti.h1, ti.h2)
    int64_t l = 0, r = n_trip;
    while (l < r) {
        const int64_t m = l + (r - l) / 2;
        const bool less = T[m].h0 < ti.h1 || (T[m].h0 == ti.h1 && T[m].h1 < ti.h2);
        if (less)
            l = m + 1;
        else
            r = m;
    }
    int64_t c = 0;
    int64_t at = FILL ? off[i] : 0;
    for (int64_t j = l; j < n_trip && T[j].h0 == ti.h1 && T[j].h1 == ti.h2; ++j) {
        const GTrip tj = T[j];
        const double dk = fabs(ti.kappa - tj.kappa);
        if (!(dk <= C.dcurv_max)) continue;
        const double hsum = 1.0 + static_cast<double>(ti.holes) + static_cast<double>(tj.holes);
        const double mx = ti.dtheta < tj.dtheta ? tj.dtheta : ti.dtheta;
        const double s = (1.0 - 0.5 * (dk + mx)) / (hsum * hsum);
        if (!(s > C.s_min)) continue;
        if (FILL) {
            qi[at] = static_cast<int32_t>(i);
            qj[at] = static_cast<int32_t>(j);
            qs[at] = s;
            ++at;
        }
        ++c;
    }
    if (!FILL) cnt[i] = c;
}

__global__ void mark_quads(int64_t n, const int32_t *__restrict__ qi, const int32_t *__restrict__ qj,
                           uint8_t *__restrict__ has_out, uint8_t *__restrict__ has_in) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kTPB + threadIdx.x;
    if (k >= n) return;
    has_out[qi[k]] = 1;
    has_in[qj[k]] = 1;
}

// keep[k] = 1 for quadruplets kept by the five-hit rule (or all of them)
__global__ void five_hit(int64_t n, int32_t rule, const int32_t *__restrict__ qi,
                         const int32_t *__restrict__ qj, const uint8_t *__restrict__ has_out,
                         const uint8_t *__restrict__ has_in, int64_t *__restrict__ keep) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kTPB + threadIdx.x;
    if (k >= n) return;
    keep[k] = (!rule || has_out[qj[k]] || has_in[qi[k]]) ? 1 : 0;
}

// compacts kept quadruplets (order kept) and marks their triplets alive
__global__ void compact_quads(int64_t n, const int64_t *__restrict__ keep,
                              const int64_t *__restrict__ pos, const int32_t *__restrict__ qi,
                              const int32_t *__restrict__ qj, const double *__restrict__ qs,
                              int32_t *__restrict__ ki, int32_t *__restrict__ kj,
                              double *__restrict__ ks, int64_t *__restrict__ alive) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kTPB + threadIdx.x;
    if (k >= n || !keep[k]) return;
    const int64_t p = pos[k];
    ki[p] = qi[k];
    kj[p] = qj[k];
    ks[p] = qs[k];
    alive[qi[k]] = 1;  // plain stores of the same value
    alive[qj[k]] = 1;
}

// surviving triplet t gets index new_id[t]; writes its bias (Eq. 15),
// hit ids and hit indices
__global__ void survivors(int64_t n_trip, const int64_t *__restrict__ alive,
                          const int64_t *__restrict__ new_id, const GTrip *__restrict__ T,
                          const int64_t *__restrict__ hit_id, Cuts C, double *__restrict__ a,
                          int64_t *__restrict__ trip_ids, int32_t *__restrict__ th) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * kTPB + threadIdx.x;
    if (t >= n_trip || !alive[t]) return;
    const int64_t k = new_id[t];
    const GTrip g = T[t];
    a[k] = C.alpha * (1.0 - exp(-fabs(g.d0) / C.gamma_)) +
           C.beta * (1.0 - exp(-fabs(g.z0) / C.lambda_));
    trip_ids[3 * k + 0] = hit_id[g.h0];
    trip_ids[3 * k + 1] = hit_id[g.h1];
    trip_ids[3 * k + 2] = hit_id[g.h2];
    th[3 * k + 0] = g.h0;
    th[3 * k + 1] = g.h1;
    th[3 * k + 2] = g.h2;
}

// ------------------------------------------------------------ conflicts

// Two triplets share a hit and are not shifted windows of one hit chain.
__device__ __forceinline__ bool conflict(const int32_t *p, const int32_t *q) {
    bool share = false;
    for (int s = 0; s < 3; ++s)
        for (int u = 0; u < 3; ++u) share |= (p[s] == q[u]);
    if (!share) return false;
    if ((p[1] == q[0] && p[2] == q[1]) || (q[1] == p[0] && q[2] == p[1])) return false;
    if (p[2] == q[0] || q[2] == p[0]) return false;
    return true;
}

__global__ void memberships(int64_t n, const int32_t *__restrict__ th, uint64_t *__restrict__ keys) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kTPB + threadIdx.x;
    if (k >= n) return;
    for (int s = 0; s < 3; ++s)
        keys[3 * k + s] = (static_cast<uint64_t>(th[3 * k + s]) << 32) | static_cast<uint32_t>(k);
}

template <bool FILL>
__global__ void conflicts_kernel(int64_t n_memb, const uint64_t *__restrict__ memb,
                                 const int32_t *__restrict__ th, int64_t *__restrict__ cnt,
                                 const int64_t *__restrict__ off, uint64_t *__restrict__ out) {
    const int64_t u = static_cast<int64_t>(blockIdx.x) * kTPB + threadIdx.x;
    if (u >= n_memb) return;
    const uint32_t hit = static_cast<uint32_t>(memb[u] >> 32);
    const int32_t tu = static_cast<int32_t>(memb[u] & 0xFFFFFFFFu);
    int64_t c = 0;
    int64_t at = FILL ? off[u] : 0;
    for (int64_t v = u + 1; v < n_memb && static_cast<uint32_t>(memb[v] >> 32) == hit; ++v) {
        const int32_t tv = static_cast<int32_t>(memb[v] & 0xFFFFFFFFu);
        if (!conflict(th + 3 * static_cast<int64_t>(tu), th + 3 * static_cast<int64_t>(tv))) continue;
        if (FILL) {
            const uint32_t lo = static_cast<uint32_t>(tu < tv ? tu : tv);
            const uint32_t hi = static_cast<uint32_t>(tu < tv ? tv : tu);
            out[at++] = (static_cast<uint64_t>(lo) << 32) | hi;
        }
        ++c;
    }
    if (!FILL) cnt[u] = c;
}

__global__ void first_of_run(int64_t n, const uint64_t *__restrict__ keys, int64_t *__restrict__ flag) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kTPB + threadIdx.x;
    if (k >= n) return;
    flag[k] = (k == 0 || keys[k] != keys[k - 1]) ? 1 : 0;
}

__global__ void scatter_runs(int64_t n, const uint64_t *__restrict__ keys, const int64_t *__restrict__ flag,
                             const int64_t *__restrict__ pos, uint64_t *__restrict__ out) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kTPB + threadIdx.x;
    if (k >= n || !flag[k]) return;
    out[pos[k]] = keys[k];
}

// -------------------------------------------------------------- CSR

// couplings: kept quadruplets (u, v, -s) then unique conflicts (u, v, +1)
__device__ __forceinline__ void coupling_at(int64_t c, int64_t n_quad, const int32_t *ki,
                                            const int32_t *kj, const double *ks,
                                            const int64_t *new_id, const uint64_t *conf,
                                            int32_t &u, int32_t &v, double &w) {
    if (c < n_quad) {
        const int32_t p = static_cast<int32_t>(new_id[ki[c]]);
        const int32_t q = static_cast<int32_t>(new_id[kj[c]]);
        u = p < q ? p : q;
        v = p < q ? q : p;
        w = -ks[c];
    } else {
        const uint64_t key = conf[c - n_quad];
        u = static_cast<int32_t>(key >> 32);
        v = static_cast<int32_t>(key & 0xFFFFFFFFu);
        w = 1.0;
    }
}

__global__ void csr_count(int64_t n_cpl, int64_t n_quad, const int32_t *ki, const int32_t *kj,
                          const double *ks, const int64_t *new_id, const uint64_t *conf,
                          int64_t *__restrict__ cnt) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kTPB + threadIdx.x;
    if (c >= n_cpl) return;
    int32_t u, v;
    double w;
    coupling_at(c, n_quad, ki, kj, ks, new_id, conf, u, v, w);
    atomicAdd(reinterpret_cast<unsigned long long *>(cnt + u), 1ull);
    atomicAdd(reinterpret_cast<unsigned long long *>(cnt + v), 1ull);
}

__global__ void csr_fill(int64_t n_cpl, int64_t n_quad, const int32_t *ki, const int32_t *kj,
                         const double *ks, const int64_t *new_id, const uint64_t *conf,
                         unsigned long long *__restrict__ cursor, int32_t *__restrict__ col,
                         double *__restrict__ b) {
    const int64_t c = static_cast<int64_t>(blockIdx.x) * kTPB + threadIdx.x;
    if (c >= n_cpl) return;
    int32_t u, v;
    double w;
    coupling_at(c, n_quad, ki, kj, ks, new_id, conf, u, v, w);
    const unsigned long long pu = atomicAdd(cursor + u, 1ull);
    col[pu] = v;
    b[pu] = w;
    const unsigned long long pv = atomicAdd(cursor + v, 1ull);
    col[pv] = u;
    b[pv] = w;
}

__global__ void csr_sort_rows(int64_t n, const int64_t *__restrict__ row_ptr, int32_t *__restrict__ col,
                              double *__restrict__ b) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * kTPB + threadIdx.x;
    if (r >= n) return;
    const int64_t s = row_ptr[r], e = row_ptr[r + 1];
    for (int64_t i = s + 1; i < e; ++i) {  // insertion sort, columns unique
        const int32_t cv = col[i];
        const double bv = b[i];
        int64_t j = i - 1;
        while (j >= s && col[j] > cv) {
            col[j + 1] = col[j];
            b[j + 1] = b[j];
            --j;
        }
        col[j + 1] = cv;
        b[j + 1] = bv;
    }
}

// ---------------------------------------------------------- host side

struct Builder {
    hipStream_t st = nullptr;
    const char *who = "sbt_build_qubo_gpu";
    int err = SBT_OK;

    bool ok(hipError_t e, const char *what) {
        if (e == hipSuccess) return true;
        err = sbt::fail(SBT_EDEVICE, "%s: %s: %s", who, what, hipGetErrorString(e));
        return false;
    }

    // out[0..n] = exclusive sum of in[0..n) with out[n] = total; in has n+1
    // entries, the last one zero
    bool exclusive(const int64_t *in, int64_t *out, int64_t n, int64_t *total) {
        size_t tmp = 0;
        if (!ok(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp, in, out, static_cast<int>(n + 1), st),
                "scan size"))
            return false;
        DArr<char> t;
        if (!ok(t.alloc(static_cast<int64_t>(tmp)), "scan storage")) return false;
        if (!ok(hipcub::DeviceScan::ExclusiveSum(t.p, tmp, in, out, static_cast<int>(n + 1), st), "scan"))
            return false;
        return ok(hipMemcpyAsync(total, out + n, sizeof(int64_t), hipMemcpyDeviceToHost, st), "scan total") &&
               ok(hipStreamSynchronize(st), "scan sync");
    }

    bool sort_keys(DArr<uint64_t> &keys, int64_t n) {
        if (n <= 1) return true;
        DArr<uint64_t> outk;
        if (!ok(outk.alloc(n), "sort buffer")) return false;
        size_t tmp = 0;
        if (!ok(hipcub::DeviceRadixSort::SortKeys(nullptr, tmp, keys.p, outk.p, static_cast<int>(n), 0, 64, st),
                "sort size"))
            return false;
        DArr<char> t;
        if (!ok(t.alloc(static_cast<int64_t>(tmp)), "sort storage")) return false;
        if (!ok(hipcub::DeviceRadixSort::SortKeys(t.p, tmp, keys.p, outk.p, static_cast<int>(n), 0, 64, st),
                "sort"))
            return false;
        std::swap(keys.p, outk.p);
        return ok(hipStreamSynchronize(st), "sort sync");
    }

    template <class T>
    bool upload(DArr<T> &d, const std::vector<T> &h) {
        if (!ok(d.alloc(static_cast<int64_t>(h.size())), "alloc")) return false;
        if (h.empty()) return true;
        return ok(hipMemcpyAsync(d.p, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, st), "upload");
    }

    template <class T>
    bool zeros(DArr<T> &d, int64_t n) {
        return ok(d.alloc(n), "alloc") &&
               ok(hipMemsetAsync(d.p, 0, sizeof(T) * static_cast<size_t>(std::max<int64_t>(n, 1)), st), "memset");
    }

    bool fits(int64_t v, const char *what) {
        if (v <= INT32_MAX / 2) return true;
        err = sbt::fail(SBT_EUNSUPPORTED, "%s: %lld %s exceed 32-bit indexing", who,
                        static_cast<long long>(v), what);
        return false;
    }

    int run(const sbt_hit *hits, int64_t n_hits, const sbt_build_params &p, sbt_qubo **out,
            double *elapsed);
};

template <class T>
T *host_copy(const DArr<T> &d, int64_t n, hipStream_t st, bool &good) {
    T *h = static_cast<T *>(std::malloc(sizeof(T) * static_cast<size_t>(std::max<int64_t>(n, 1))));
    if (!h) throw std::bad_alloc();
    if (n > 0 && hipMemcpyAsync(h, d.p, sizeof(T) * static_cast<size_t>(n), hipMemcpyDeviceToHost, st) != hipSuccess)
        good = false;
    return h;
}

int Builder::run(const sbt_hit *hits, int64_t n_hits, const sbt_build_params &p, sbt_qubo **out,
                 double *elapsed) {
    // ---- host prelude: hits by id, layers, azimuth-sorted layer lists
    std::vector<int64_t> order(static_cast<size_t>(n_hits));
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(),
              [&](int64_t u, int64_t v) { return hits[u].hit_id < hits[v].hit_id; });
    std::vector<double> hx(n_hits), hy(n_hits), hz(n_hits), hphi(n_hits);
    std::vector<int32_t> hlayer(n_hits);
    std::vector<int64_t> hid(n_hits);
    int32_t n_layers = 0;
    for (int64_t k = 0; k < n_hits; ++k) {
        const sbt_hit &h = hits[order[k]];
        if (k > 0 && h.hit_id == hid[k - 1])
            return sbt::fail(SBT_EINVAL, "%s: duplicate hit id %lld", who, static_cast<long long>(h.hit_id));
        hid[k] = h.hit_id;
        hlayer[k] = h.layer;
        hx[k] = h.x;
        hy[k] = h.y;
        hz[k] = h.z;
        hphi[k] = std::atan2(h.y, h.x);
        n_layers = std::max(n_layers, h.layer + 1);
    }
    const int32_t mth = p.min_track_hits >= 0 ? p.min_track_hits : std::min(5, n_layers);
    if (mth > 5) return sbt::fail(SBT_EUNSUPPORTED, "%s: min_track_hits > 5 not implemented", who);
    // per layer: hits in azimuth order (ties by index); inner hits in id order
    std::vector<int32_t> lay_off(static_cast<size_t>(n_layers) + 2, 0), phi_idx(n_hits), inner;
    std::vector<double> phi_val(n_hits);
    for (int64_t k = 0; k < n_hits; ++k) lay_off[hlayer[k] + 1]++;
    for (int32_t L = 0; L < n_layers; ++L) lay_off[L + 1] += lay_off[L];
    lay_off[n_layers + 1] = lay_off[n_layers];
    {
        std::vector<int32_t> fill(lay_off.begin(), lay_off.end() - 1);
        for (int32_t k = 0; k < static_cast<int32_t>(n_hits); ++k) phi_idx[fill[hlayer[k]]++] = k;
        for (int32_t L = 0; L < n_layers; ++L)
            std::sort(phi_idx.begin() + lay_off[L], phi_idx.begin() + lay_off[L + 1],
                      [&](int32_t u, int32_t v) { return hphi[u] < hphi[v] || (hphi[u] == hphi[v] && u < v); });
        for (int64_t q = 0; q < n_hits; ++q) phi_val[q] = hphi[phi_idx[q]];
        for (int32_t k = 0; k < static_cast<int32_t>(n_hits); ++k)
            if (hlayer[k] + 1 < n_layers) inner.push_back(k);
    }
    Cuts C;
    C.dphi_tan = p.dphi_tan;
    C.z0_max = p.z0_max;
    C.curv_max = p.curv_max;
    C.dtheta_tan = p.dtheta_tan;
    C.dcurv_max = p.dcurv_max;
    C.s_min = p.s_min;
    C.alpha = p.alpha;
    C.beta = p.beta;
    C.gamma_ = p.gamma_;
    C.lambda_ = p.lambda_;
    C.win = std::atan(p.dphi_tan) + 1e-6;
    C.all = !(C.win < 0.5 * kPi) ? 1 : 0;
    C.max_holes = p.max_holes;

    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!ok(hipEventCreate(&e0), "event") || !ok(hipEventCreate(&e1), "event")) return err;
    struct EvGuard {
        hipEvent_t a, b;
        ~EvGuard() {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } evg{e0, e1};

    DArr<double> dx, dy, dz, dphi, dphival;
    DArr<int32_t> dlayer, dlayoff, dphiidx, dinner;
    DArr<int64_t> did;
    if (!upload(dx, hx) || !upload(dy, hy) || !upload(dz, hz) || !upload(dphi, hphi) ||
        !upload(dphival, phi_val) || !upload(dlayer, hlayer) || !upload(dlayoff, lay_off) ||
        !upload(dphiidx, phi_idx) || !upload(dinner, inner) || !upload(did, hid))
        return err;
    if (!ok(hipEventRecord(e0, st), "event")) return err;
    const Geo G{dx.p, dy.p, dz.p, dphi.p, dlayer.p};
    const int64_t n_inner = static_cast<int64_t>(inner.size());

    // ---- 1. doublets, sorted by (inner, outer)
    DArr<int64_t> cnt, off;
    int64_t n_dbl = 0;
    if (!zeros(cnt, n_inner + 1) || !ok(off.alloc(n_inner + 1), "alloc")) return err;
    if (n_inner > 0)
        doublets_kernel<false><<<blocks(n_inner), kTPB, 0, st>>>(n_inner, dinner.p, G, C, dlayoff.p, dphiidx.p,
                                                                 dphival.p, cnt.p, nullptr, nullptr);
    if (!ok(hipGetLastError(), "doublet count") || !exclusive(cnt.p, off.p, n_inner, &n_dbl) ||
        !fits(n_dbl, "doublets"))
        return err;
    DArr<uint64_t> dkeys;
    if (!ok(dkeys.alloc(n_dbl), "alloc")) return err;
    if (n_inner > 0)
        doublets_kernel<true><<<blocks(n_inner), kTPB, 0, st>>>(n_inner, dinner.p, G, C, dlayoff.p, dphiidx.p,
                                                                dphival.p, nullptr, off.p, dkeys.p);
    if (!ok(hipGetLastError(), "doublet fill") || !sort_keys(dkeys, n_dbl)) return err;
    DArr<int32_t> din, dout;
    if (!ok(din.alloc(n_dbl), "alloc") || !ok(dout.alloc(n_dbl), "alloc")) return err;
    if (n_dbl > 0) decode_pairs<<<blocks(n_dbl), kTPB, 0, st>>>(n_dbl, dkeys.p, din.p, dout.p);
    // outgoing adjacency over hits
    DArr<int64_t> hcnt, out_ptr;
    int64_t tot = 0;
    if (!zeros(hcnt, n_hits + 1) || !ok(out_ptr.alloc(n_hits + 1), "alloc")) return err;
    if (n_dbl > 0) count_first<<<blocks(n_dbl), kTPB, 0, st>>>(n_dbl, din.p, hcnt.p);
    if (!ok(hipGetLastError(), "adjacency") || !exclusive(hcnt.p, out_ptr.p, n_hits, &tot)) return err;

    // ---- 2. triplets in (h1, h2, h3) order
    DArr<int64_t> tcnt, toff;
    int64_t n_trip = 0;
    if (!zeros(tcnt, n_dbl + 1) || !ok(toff.alloc(n_dbl + 1), "alloc")) return err;
    if (n_dbl > 0)
        triplets_kernel<false><<<blocks(n_dbl), kTPB, 0, st>>>(n_dbl, din.p, dout.p, out_ptr.p, G, C, tcnt.p,
                                                               nullptr, nullptr);
    if (!ok(hipGetLastError(), "triplet count") || !exclusive(tcnt.p, toff.p, n_dbl, &n_trip) ||
        !fits(n_trip, "triplets"))
        return err;
    DArr<GTrip> trips;
    if (!ok(trips.alloc(n_trip), "alloc")) return err;
    if (n_dbl > 0)
        triplets_kernel<true><<<blocks(n_dbl), kTPB, 0, st>>>(n_dbl, din.p, dout.p, out_ptr.p, G, C, nullptr,
                                                              toff.p, trips.p);
    if (!ok(hipGetLastError(), "triplet fill")) return err;

    // ---- 3. quadruplets (Eq. 14, 17)
    DArr<int64_t> qcnt, qoff;
    int64_t n_q = 0;
    if (!zeros(qcnt, n_trip + 1) || !ok(qoff.alloc(n_trip + 1), "alloc")) return err;
    if (n_trip > 0)
        quads_kernel<false><<<blocks(n_trip), kTPB, 0, st>>>(n_trip, trips.p, C, qcnt.p, nullptr, nullptr,
                                                             nullptr, nullptr);
    if (!ok(hipGetLastError(), "quad count") || !exclusive(qcnt.p, qoff.p, n_trip, &n_q) ||
        !fits(n_q, "quadruplets"))
        return err;
    DArr<int32_t> qi, qj;
    DArr<double> qs;
    if (!ok(qi.alloc(n_q), "alloc") || !ok(qj.alloc(n_q), "alloc") || !ok(qs.alloc(n_q), "alloc")) return err;
    if (n_trip > 0)
        quads_kernel<true><<<blocks(n_trip), kTPB, 0, st>>>(n_trip, trips.p, C, nullptr, qoff.p, qi.p, qj.p,
                                                            qs.p);
    if (!ok(hipGetLastError(), "quad fill")) return err;

    // ---- 4. five-hit rule; 5. surviving triplets
    DArr<uint8_t> has_out, has_in;
    DArr<int64_t> keep, kpos, alive, new_id;
    int64_t n_kept = 0, n = 0;
    if (!zeros(has_out, n_trip) || !zeros(has_in, n_trip) || !zeros(keep, n_q + 1) ||
        !ok(kpos.alloc(n_q + 1), "alloc") || !zeros(alive, n_trip + 1) || !ok(new_id.alloc(n_trip + 1), "alloc"))
        return err;
    if (n_q > 0) {
        mark_quads<<<blocks(n_q), kTPB, 0, st>>>(n_q, qi.p, qj.p, has_out.p, has_in.p);
        five_hit<<<blocks(n_q), kTPB, 0, st>>>(n_q, mth >= 5 ? 1 : 0, qi.p, qj.p, has_out.p, has_in.p, keep.p);
    }
    if (!ok(hipGetLastError(), "five-hit rule") || !exclusive(keep.p, kpos.p, n_q, &n_kept)) return err;
    DArr<int32_t> ki, kj;
    DArr<double> ks;
    if (!ok(ki.alloc(n_kept), "alloc") || !ok(kj.alloc(n_kept), "alloc") || !ok(ks.alloc(n_kept), "alloc"))
        return err;
    if (n_q > 0)
        compact_quads<<<blocks(n_q), kTPB, 0, st>>>(n_q, keep.p, kpos.p, qi.p, qj.p, qs.p, ki.p, kj.p, ks.p,
                                                    alive.p);
    if (!ok(hipGetLastError(), "compact") || !exclusive(alive.p, new_id.p, n_trip, &n)) return err;

    // ---- 6. biases (Eq. 15) and hit ids of the survivors
    DArr<double> da;
    DArr<int64_t> dtrip_ids;
    DArr<int32_t> dth;
    if (!ok(da.alloc(n), "alloc") || !ok(dtrip_ids.alloc(3 * n), "alloc") || !ok(dth.alloc(3 * n), "alloc"))
        return err;
    if (n_trip > 0)
        survivors<<<blocks(n_trip), kTPB, 0, st>>>(n_trip, alive.p, new_id.p, trips.p, did.p, C, da.p,
                                                   dtrip_ids.p, dth.p);
    if (!ok(hipGetLastError(), "survivors")) return err;

    // ---- 7. conflicts: pairs of survivors sharing a hit
    DArr<uint64_t> memb;
    const int64_t n_memb = 3 * n;
    if (!ok(memb.alloc(n_memb), "alloc")) return err;
    if (n > 0) memberships<<<blocks(n), kTPB, 0, st>>>(n, dth.p, memb.p);
    if (!ok(hipGetLastError(), "memberships") || !sort_keys(memb, n_memb)) return err;
    DArr<int64_t> ccnt, coff;
    int64_t n_c = 0;
    if (!zeros(ccnt, n_memb + 1) || !ok(coff.alloc(n_memb + 1), "alloc")) return err;
    if (n_memb > 0)
        conflicts_kernel<false><<<blocks(n_memb), kTPB, 0, st>>>(n_memb, memb.p, dth.p, ccnt.p, nullptr,
                                                                 nullptr);
    if (!ok(hipGetLastError(), "conflict count") || !exclusive(ccnt.p, coff.p, n_memb, &n_c) ||
        !fits(n_c, "conflict pairs"))
        return err;
    DArr<uint64_t> conf;
    if (!ok(conf.alloc(n_c), "alloc")) return err;
    if (n_memb > 0)
        conflicts_kernel<true><<<blocks(n_memb), kTPB, 0, st>>>(n_memb, memb.p, dth.p, nullptr, coff.p,
                                                                conf.p);
    if (!ok(hipGetLastError(), "conflict fill") || !sort_keys(conf, n_c)) return err;
    DArr<int64_t> uflag, upos;
    int64_t n_u = 0;
    if (!zeros(uflag, n_c + 1) || !ok(upos.alloc(n_c + 1), "alloc")) return err;
    if (n_c > 0) first_of_run<<<blocks(n_c), kTPB, 0, st>>>(n_c, conf.p, uflag.p);
    if (!ok(hipGetLastError(), "unique") || !exclusive(uflag.p, upos.p, n_c, &n_u)) return err;
    DArr<uint64_t> uconf;
    if (!ok(uconf.alloc(n_u), "alloc")) return err;
    if (n_c > 0) scatter_runs<<<blocks(n_c), kTPB, 0, st>>>(n_c, conf.p, uflag.p, upos.p, uconf.p);
    if (!ok(hipGetLastError(), "unique scatter")) return err;

    // ---- 8. symmetric CSR, ascending columns
    const int64_t n_cpl = n_kept + n_u;
    if (!fits(2 * n_cpl, "stored couplings")) return err;
    DArr<int64_t> rcnt, row_ptr;
    int64_t nnz = 0;
    if (!zeros(rcnt, n + 1) || !ok(row_ptr.alloc(n + 1), "alloc")) return err;
    if (n_cpl > 0)
        csr_count<<<blocks(n_cpl), kTPB, 0, st>>>(n_cpl, n_kept, ki.p, kj.p, ks.p, new_id.p, uconf.p, rcnt.p);
    if (!ok(hipGetLastError(), "csr count") || !exclusive(rcnt.p, row_ptr.p, n, &nnz)) return err;
    DArr<unsigned long long> cursor;
    DArr<int32_t> dcol;
    DArr<double> db;
    if (!ok(cursor.alloc(n + 1), "alloc") || !ok(dcol.alloc(nnz), "alloc") || !ok(db.alloc(nnz), "alloc"))
        return err;
    if (!ok(hipMemcpyAsync(cursor.p, row_ptr.p, sizeof(int64_t) * static_cast<size_t>(n + 1),
                           hipMemcpyDeviceToDevice, st), "cursor"))
        return err;
    if (n_cpl > 0)
        csr_fill<<<blocks(n_cpl), kTPB, 0, st>>>(n_cpl, n_kept, ki.p, kj.p, ks.p, new_id.p, uconf.p, cursor.p,
                                                dcol.p, db.p);
    if (n > 0) csr_sort_rows<<<blocks(n), kTPB, 0, st>>>(n, row_ptr.p, dcol.p, db.p);
    if (!ok(hipGetLastError(), "csr fill") || !ok(hipEventRecord(e1, st), "event") ||
        !ok(hipStreamSynchronize(st), "sync"))
        return err;
    if (elapsed) {
        float ms = 0.0f;
        if (!ok(hipEventElapsedTime(&ms, e0, e1), "event time")) return err;
        *elapsed = ms * 1e-3;
    }

    // ---- download into a library-owned QUBO
    sbt_qubo *q = static_cast<sbt_qubo *>(std::calloc(1, sizeof(sbt_qubo)));
    if (!q) throw std::bad_alloc();
    q->n = static_cast<int32_t>(n);
    q->nnz = nnz;
    bool good = true;
    try {
        q->a = host_copy(da, n, st, good);
        q->row_ptr = host_copy(row_ptr, n + 1, st, good);
        q->col = host_copy(dcol, nnz, st, good);
        q->b = host_copy(db, nnz, st, good);
        q->trip_hits = host_copy(dtrip_ids, 3 * n, st, good);
    } catch (...) {
        sbt_qubo_free(q);
        throw;
    }
    if (n == 0) q->row_ptr[0] = 0;
    if (!good || !ok(hipStreamSynchronize(st), "download")) {
        sbt_qubo_free(q);
        if (good) return err;
        return sbt::fail(SBT_EDEVICE, "%s: download failed", who);
    }
    *out = q;
    return SBT_OK;
}

}  // namespace

extern "C" int sbt_build_qubo_gpu(const sbt_hit *hits, int64_t n_hits, const sbt_build_params *pp,
                                  sbt_qubo **out, double *elapsed_s) {
    sbt::clear_error();
    sbt_build_params p;
    const int rc = sbt::check_build_inputs(hits, n_hits, pp, out, &p, "sbt_build_qubo_gpu");
    if (rc) return rc;
    if (elapsed_s) *elapsed_s = 0.0;
    Builder B;
    if (hipStreamCreateWithFlags(&B.st, hipStreamNonBlocking) != hipSuccess)
        return sbt::fail(SBT_EDEVICE, "sbt_build_qubo_gpu: no HIP stream");
    int r;
    try {
        r = B.run(hits, n_hits, p, out, elapsed_s);
    } catch (const std::bad_alloc &) {
        r = sbt::fail(SBT_ENOMEM, "sbt_build_qubo_gpu: out of host memory");
    }
    (void)hipStreamDestroy(B.st);
    return r;
}
