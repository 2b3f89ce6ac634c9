// Driver for the sanitizer builds of the library's host code (test
// infrastructure).  Built with g++ together with the host sources only
// (status, validate, build_qubo, order, anneal: no HIP), under
// AddressSanitizer + UndefinedBehaviorSanitizer or ThreadSanitizer, by
// tests/test_sanitize_cpu.py.
//
//   host_abi_check EVENTS OUT
//
// EVENTS: a sequence of events, each int64 n_hits followed by n_hits
// sbt_hit records.  For every event the driver builds the QUBO, orders and
// relabels it, evaluates O(T) for a fixed T and anneals it briefly on two
// threads, writing everything to OUT (the test compares OUT with the
// regular library's results).  It then feeds malformed inputs to every
// entry point and checks each is refused with SBT_EINVAL; any other
// status, or any sanitizer report, fails the run.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "sbtrack.h"

namespace {

int g_fail = 0;

void expect(bool ok, const char *what) {
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s (%s)\n", what, sbt_last_error());
        g_fail = 1;
    }
}

template <class T>
void put(std::FILE *f, const T *p, size_t n) {
    if (n && std::fwrite(p, sizeof(T), n, f) != n) {
        std::fprintf(stderr, "write failed\n");
        std::exit(2);
    }
}

void run_event(const std::vector<sbt_hit> &hits, std::FILE *out) {
    sbt_qubo *q = nullptr;
    const int rc = sbt_build_qubo(hits.data(), static_cast<int64_t>(hits.size()), nullptr, &q);
    expect(rc == SBT_OK, "sbt_build_qubo");
    if (rc) return;
    put(out, &q->n, 1);
    put(out, &q->nnz, 1);
    put(out, q->a, q->n);
    put(out, q->row_ptr, static_cast<size_t>(q->n) + 1);
    put(out, q->col, q->nnz);
    put(out, q->b, q->nnz);
    put(out, q->trip_hits, 3 * static_cast<size_t>(q->n));
    if (q->n > 0) {
        int32_t mr = -1;
        expect(sbt::validate_qubo_host(q, "check", "qubo", &mr) == SBT_OK, "valid QUBO accepted");
        std::vector<int32_t> perm(q->n);
        expect(sbt_phi_order(q, hits.data(), static_cast<int64_t>(hits.size()), perm.data()) ==
                   SBT_OK,
               "sbt_phi_order");
        put(out, perm.data(), perm.size());
        sbt_qubo *qp = nullptr;
        expect(sbt_qubo_permute(q, perm.data(), &qp) == SBT_OK, "sbt_qubo_permute");
        if (qp) {
            put(out, qp->row_ptr, static_cast<size_t>(qp->n) + 1);
            put(out, qp->col, qp->nnz);
            put(out, qp->b, qp->nnz);
            sbt_qubo_free(qp);
        }
        std::vector<int8_t> T(q->n);
        for (int32_t i = 0; i < q->n; ++i) T[i] = static_cast<int8_t>((i * 7 + 3) % 5 < 2);
        double e = 0.0;
        expect(sbt_energy(q, T.data(), &e) == SBT_OK, "sbt_energy");
        put(out, &e, 1);
        sbt_anneal_params ap;
        sbt_anneal_params_default(&ap);
        ap.shots = 6;
        ap.sweeps = 20;
        ap.threads = 2;
        ap.seed = 11;
        std::vector<int8_t> Tb(q->n);
        std::vector<double> se(ap.shots);
        double eb = 0.0;
        expect(sbt_anneal_cpu(q, &ap, Tb.data(), &eb, se.data(), nullptr) == SBT_OK,
               "sbt_anneal_cpu");
        put(out, se.data(), se.size());
    }
    sbt_qubo_free(q);
}

// A well-formed 3-variable QUBO: b_01 = b_10 = 1, b_12 = b_21 = -0.5.
struct Small {
    double a[3] = {0.1, 0.2, 0.3};
    int64_t rp[4] = {0, 1, 3, 4};
    int32_t col[4] = {1, 0, 2, 1};
    double b[4] = {1.0, 1.0, -0.5, -0.5};
    int64_t th[9] = {0, 1, 2, 1, 2, 3, 2, 3, 4};
    sbt_qubo q() { return sbt_qubo{3, 4, a, rp, col, b, th}; }
};

void negative_cases() {
    Small s;
    sbt_qubo q = s.q();
    expect(sbt::validate_qubo_host(&q, "check", "qubo", nullptr) == SBT_OK, "small QUBO valid");
    auto refused = [&](sbt_qubo bad, const char *what) {
        expect(sbt::validate_qubo_host(&bad, "check", "qubo", nullptr) == SBT_EINVAL, what);
        int8_t T[8] = {0};
        double e = 0.0;
        sbt_anneal_params ap;
        sbt_anneal_params_default(&ap);
        ap.shots = 2;
        ap.sweeps = 2;
        ap.threads = 1;
        if (bad.n > 0 && bad.n <= 8)
            expect(sbt_anneal_cpu(&bad, &ap, T, &e, nullptr, nullptr) == SBT_EINVAL, what);
    };
    {  // row pointers that decrease, leave [0, nnz] or do not span it
        int64_t rp1[4] = {0, 3, 1, 4};
        sbt_qubo b = q;
        b.row_ptr = rp1;
        refused(b, "decreasing row_ptr");
        int64_t rp2[4] = {0, 9, 2, 4};
        b.row_ptr = rp2;
        refused(b, "row_ptr past nnz");
        int64_t rp3[4] = {0, -1, 3, 4};
        b.row_ptr = rp3;
        refused(b, "negative row_ptr");
        int64_t rp4[4] = {0, 1, 3, 3};
        b.row_ptr = rp4;
        refused(b, "row_ptr not ending at nnz");
    }
    {  // columns out of range, unsorted, on the diagonal; asymmetric b; NaN
        int32_t c1[4] = {1, 0, 7, 1};
        sbt_qubo b = q;
        b.col = c1;
        refused(b, "column out of range");
        int32_t c2[4] = {1, 2, 0, 1};
        b.col = c2;
        refused(b, "columns not ascending");
        int32_t c3[4] = {0, 0, 2, 1};
        b.col = c3;
        refused(b, "diagonal entry");
        double b1[4] = {1.0, 0.5, -0.5, -0.5};
        sbt_qubo bb = q;
        bb.b = b1;
        refused(bb, "asymmetric b");
        double a1[3] = {0.1, NAN, 0.3};
        sbt_qubo ba = q;
        ba.a = a1;
        refused(ba, "NaN bias");
        sbt_qubo bn = q;
        bn.n = 0;
        refused(bn, "empty QUBO");
    }
    {  // construction: bad hit arrays
        sbt_hit h[3] = {{1, 0, 0, 10.0, 0.0, 0.0}, {1, 1, 0, 20.0, 0.0, 0.0},
                        {3, 2, 0, 30.0, 0.0, 0.0}};
        sbt_qubo *out = nullptr;
        expect(sbt_build_qubo(h, 3, nullptr, &out) == SBT_EINVAL, "duplicate hit ids");
        h[1].hit_id = 2;
        h[2].x = NAN;
        expect(sbt_build_qubo(h, 3, nullptr, &out) == SBT_EINVAL, "NaN coordinate");
        h[2].x = 30.0;
        h[2].layer = -1;
        expect(sbt_build_qubo(h, 3, nullptr, &out) == SBT_EINVAL, "negative layer");
        expect(sbt_build_qubo(h, -1, nullptr, &out) == SBT_EINVAL, "negative hit count");
    }
    {  // relabelling: not a permutation; ordering: triplets naming absent hits
        int32_t perm[3] = {0, 0, 2};
        sbt_qubo *out = nullptr;
        expect(sbt_qubo_permute(&q, perm, &out) == SBT_EINVAL, "repeated index in perm");
        int32_t perm2[3] = {0, 1, 3};
        expect(sbt_qubo_permute(&q, perm2, &out) == SBT_EINVAL, "index out of range in perm");
        sbt_hit h[2] = {{0, 0, 0, 1.0, 0.0, 0.0}, {1, 1, 0, 2.0, 0.0, 0.0}};
        int32_t po[3];
        expect(sbt_phi_order(&q, h, 2, po) == SBT_EINVAL, "triplet names an absent hit");
        int8_t T[3] = {0, 2, 1};
        double e = 0.0;
        expect(sbt_energy(&q, T, &e) == SBT_EINVAL, "T not 0/1");
    }
}

}  // namespace

int main(int argc, char **argv) {
    if (argc != 3) {
        std::fprintf(stderr, "usage: %s EVENTS OUT\n", argv[0]);
        return 2;
    }
    std::FILE *in = std::fopen(argv[1], "rb");
    std::FILE *out = std::fopen(argv[2], "wb");
    if (!in || !out) {
        std::fprintf(stderr, "cannot open files\n");
        return 2;
    }
    int events = 0;
    for (;;) {
        int64_t nh = 0;
        if (std::fread(&nh, sizeof nh, 1, in) != 1) break;
        if (nh < 0 || nh > (int64_t(1) << 26)) return 2;
        std::vector<sbt_hit> hits(static_cast<size_t>(nh));
        if (nh && std::fread(hits.data(), sizeof(sbt_hit), hits.size(), in) != hits.size()) return 2;
        run_event(hits, out);
        ++events;
    }
    negative_cases();
    std::fclose(in);
    std::fclose(out);
    std::printf("events %d, %s\n", events, g_fail ? "FAILED" : "ok");
    return g_fail;
}
