// Single-flip Metropolis simulated annealing on the CPU: the comparator of
// the paper's section "Simulated Annealing" (a random single-spin move,
// accepted if it lowers the energy, else with probability exp(-dE / kT),
// while the temperature falls), written from that description.
//
// Readings where the paper defers to its reference solver:
//   * moves: sweeps over the spins in index order, one flip attempt each;
//   * schedule: inverse temperature geometric from beta_hot to beta_cold over
//     the sweeps; by default beta_hot accepts the largest possible energy
//     rise with probability 1/2 and beta_cold the smallest nonzero
//     coefficient's rise with probability 1/100;
//   * energy: the QUBO objective O(T) of Eq. 13 directly (flip i changes it
//     by (1 - 2 T_i)(a_i + sum_j b_ij T_j)), FP64, local fields updated on
//     every accepted flip; the reported energies are recomputed from T;
//   * shots are independent (own random stream, all-zero start), run on
//     host threads.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <new>
#include <system_error>
#include <thread>
#include <vector>

#include "common.hpp"
#include "sbtrack.h"

namespace {

// splitmix64: seeds a shot's stream from (seed, shot)
uint64_t splitmix64(uint64_t &s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// xoshiro256** (Blackman and Vigna), uniform doubles in [0, 1)
struct Rng {
    uint64_t s[4];
    explicit Rng(uint64_t seed) {
        for (auto &v : s) v = splitmix64(seed);
    }
    static uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
    uint64_t next() {
        const uint64_t r = rotl(s[1] * 5, 7) * 9;
        const uint64_t t = s[1] << 17;
        s[2] ^= s[0];
        s[3] ^= s[1];
        s[1] ^= s[2];
        s[0] ^= s[3];
        s[2] ^= t;
        s[3] = rotl(s[3], 45);
        return r;
    }
    double uniform() { return static_cast<double>(next() >> 11) * 0x1.0p-53; }
};

double objective(const sbt_qubo *q, const int8_t *T) {
    double e = 0.0;
    if (sbt_energy(q, T, &e) != SBT_OK) return std::numeric_limits<double>::quiet_NaN();
    return e;
}

void anneal_shot(const sbt_qubo *q, int32_t sweeps, double b_hot, double b_cold, uint64_t seed,
                 std::vector<int8_t> &T) {
    const int32_t n = q->n;
    std::fill(T.begin(), T.end(), 0);
    std::vector<double> f(q->a, q->a + n);  // a_i + sum_j b_ij T_j
    Rng rng(seed);
    const double ratio = sweeps > 1 ? std::pow(b_cold / b_hot, 1.0 / (sweeps - 1)) : 1.0;
    double beta = b_hot;
    for (int32_t s = 0; s < sweeps; ++s, beta *= ratio) {
        for (int32_t i = 0; i < n; ++i) {
            const double dE = T[i] ? -f[i] : f[i];
            if (dE > 0.0 && !(rng.uniform() < std::exp(-beta * dE))) continue;
            const double sgn = T[i] ? -1.0 : 1.0;
            T[i] ^= 1;
            for (int64_t p = q->row_ptr[i]; p < q->row_ptr[i + 1]; ++p) f[q->col[p]] += sgn * q->b[p];
        }
    }
}

}  // namespace

extern "C" void sbt_anneal_params_default(sbt_anneal_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->shots = 50;
    p->sweeps = 1000;
    p->beta_hot = 0.0;
    p->beta_cold = 0.0;
    p->seed = 0;
    p->threads = 0;
}

extern "C" int sbt_anneal_cpu(const sbt_qubo *q, const sbt_anneal_params *pp, int8_t *T_best,
                              double *energy, double *shot_energy, double *elapsed_s) {
    const char *who = "sbt_anneal_cpu";
    sbt::clear_error();
    if (!q || !T_best || !energy) return sbt::fail(SBT_EINVAL, "%s: NULL argument", who);
    // flips update the neighbours' local fields from row i's entries, which
    // needs b symmetric as well as well formed
    const int vrc = sbt::validate_qubo_host(q, who, "qubo", nullptr);
    if (vrc) return vrc;
    sbt_anneal_params p;
    if (pp)
        p = *pp;
    else
        sbt_anneal_params_default(&p);
    if (p.shots < 1 || p.sweeps < 1 || p.threads < 0)
        return sbt::fail(SBT_EINVAL, "%s: shots and sweeps must be >= 1, threads >= 0", who);
    // default temperatures from the coefficient ranges
    double dmax = 0.0, dmin = std::numeric_limits<double>::infinity();
    for (int32_t i = 0; i < q->n; ++i) {
        double row = std::fabs(q->a[i]);
        if (q->a[i] != 0.0) dmin = std::min(dmin, std::fabs(q->a[i]));
        for (int64_t k = q->row_ptr[i]; k < q->row_ptr[i + 1]; ++k) {
            row += std::fabs(q->b[k]);
            if (q->b[k] != 0.0) dmin = std::min(dmin, std::fabs(q->b[k]));
        }
        dmax = std::max(dmax, row);
    }
    if (!(dmax > 0.0)) dmax = 1.0;
    if (!std::isfinite(dmin)) dmin = dmax;
    const double b_hot = p.beta_hot > 0.0 ? p.beta_hot : std::log(2.0) / dmax;
    const double b_cold = p.beta_cold > 0.0 ? p.beta_cold : std::log(100.0) / dmin;
    unsigned nt = p.threads > 0 ? static_cast<unsigned>(p.threads) : std::thread::hardware_concurrency();
    nt = std::max(1u, std::min(nt, static_cast<unsigned>(p.shots)));

    const auto t0 = std::chrono::steady_clock::now();
    std::vector<double> es(p.shots);
    std::vector<std::vector<int8_t>> best_T(nt, std::vector<int8_t>(q->n));
    std::vector<double> best_e(nt, std::numeric_limits<double>::infinity());
    std::vector<int32_t> best_s(nt, -1);
    // worker w runs shots w, w + nt, ...; a worker that cannot start leaves
    // its shots to the calling thread
    std::atomic<bool> oom{false};
    auto worker = [&](unsigned w) {
        try {
            std::vector<int8_t> T(q->n);
            for (int32_t s = static_cast<int32_t>(w); s < p.shots; s += static_cast<int32_t>(nt)) {
                anneal_shot(q, p.sweeps, b_hot, b_cold,
                            p.seed * 0x100000001B3ull + static_cast<uint64_t>(s), T);
                es[s] = objective(q, T.data());
                if (es[s] < best_e[w] || (es[s] == best_e[w] && s < best_s[w])) {
                    best_e[w] = es[s];
                    best_s[w] = s;
                    best_T[w] = T;
                }
            }
        } catch (const std::bad_alloc &) {
            oom = true;
        }
    };
    try {
        std::vector<std::thread> pool;
        std::vector<unsigned> inline_workers;
        pool.reserve(nt);
        inline_workers.reserve(nt);
        for (unsigned w = 1; w < nt; ++w) {
            try {
                pool.emplace_back(worker, w);
            } catch (const std::system_error &) {
                inline_workers.push_back(w);
            }
        }
        worker(0);
        for (unsigned w : inline_workers) worker(w);
        for (auto &th : pool) th.join();
    } catch (const std::bad_alloc &) {
        return sbt::fail(SBT_ENOMEM, "%s: out of host memory", who);
    }
    if (oom) return sbt::fail(SBT_ENOMEM, "%s: out of host memory", who);
    const auto t1 = std::chrono::steady_clock::now();
    unsigned wb = 0;
    for (unsigned w = 1; w < nt; ++w)
        if (best_e[w] < best_e[wb] || (best_e[w] == best_e[wb] && best_s[w] < best_s[wb])) wb = w;
    std::copy(best_T[wb].begin(), best_T[wb].end(), T_best);
    *energy = best_e[wb];
    if (shot_energy) std::copy(es.begin(), es.end(), shot_energy);
    if (elapsed_s) *elapsed_s = std::chrono::duration<double>(t1 - t0).count();
    return SBT_OK;
}
