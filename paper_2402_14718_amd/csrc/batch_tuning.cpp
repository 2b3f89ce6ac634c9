// The batch tuning cache (host, no HIP): the key of a batch and the lookup
// of the tuned schedule in the JSON file the project's tuner writes
// (paper_2402_14718_amd/autotune.py).
//
// Key: "<mode> <precision> M<agents> h=<c0>,...,<c8>", c_k the number of
// events with n in (64 * 2^(k-1), 64 * 2^k] (c_0: n <= 64; c_8: n <= 16384).
// Lookup: the entry with the same key; else, among entries of the same
// mode, precision and agents, the one whose normalised histogram is nearest
// in L1 distance, if that distance is at most 0.25; else the defaults.
//
// File (written by the tuner; only these fields are read):
//   {"format": "sbtrack batch tuning 1", "entries": [
//     {"key": "...", "split_n": 4608, "tail_words": 8192, "fill": 1.0,
//      "band_rows": 0 (optional), ...}, ...]}
#include <dlfcn.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "sbtrack.h"

namespace {

constexpr int kBuckets = 9;

struct Entry {
    std::string key, prefix;
    std::vector<double> hist;  // normalised
    sbt_batch_tuning t;
};

const char *mode_name(sbt_mode m) { return m == SBT_BSB ? "bsb" : m == SBT_DSB ? "dsb" : "asb"; }
const char *prec_name(sbt_precision p) { return p == SBT_PREC_FP16 ? "fp16" : "bf16"; }

std::string prefix_of(sbt_mode mode, sbt_precision prec, int32_t agents) {
    char b[64];
    std::snprintf(b, sizeof b, "%s %s M%d", mode_name(mode), prec_name(prec), agents);
    return b;
}

std::vector<int64_t> histogram(const int32_t *n, int32_t E) {
    std::vector<int64_t> h(kBuckets, 0);
    for (int32_t e = 0; e < E; ++e) {
        int k = 0;
        while (k < kBuckets - 1 && n[e] > (64 << k)) ++k;
        ++h[k];
    }
    return h;
}

std::string key_of(const std::string &prefix, const std::vector<int64_t> &h) {
    std::string k = prefix + " h=";
    for (int i = 0; i < kBuckets; ++i) k += (i ? "," : "") + std::to_string(h[i]);
    return k;
}

// Number after "name": inside [from, to) of s, or NaN.
double field(const std::string &s, size_t from, size_t to, const char *name) {
    const std::string pat = std::string("\"") + name + "\"";
    const size_t at = s.find(pat, from);
    if (at == std::string::npos || at >= to) return NAN;
    const size_t colon = s.find(':', at + pat.size());
    if (colon == std::string::npos || colon >= to) return NAN;
    return std::strtod(s.c_str() + colon + 1, nullptr);
}

std::string cache_path() {
    if (const char *env = std::getenv("SBT_BATCH_TUNING_CACHE")) return env;
    Dl_info info{};
    if (dladdr(reinterpret_cast<void *>(&sbt_batch_tuning_lookup), &info) && info.dli_fname) {
        std::string lib = info.dli_fname;
        const size_t slash = lib.rfind('/');
        return (slash == std::string::npos ? std::string(".") : lib.substr(0, slash)) +
               "/tuning/batch_tuning.json";
    }
    return "tuning/batch_tuning.json";
}

// Entries of the cache file, read once per process.
const std::vector<Entry> &entries() {
    static std::once_flag once;
    static std::vector<Entry> all;
    std::call_once(once, [] {
        std::FILE *f = std::fopen(cache_path().c_str(), "rb");
        if (!f) return;
        std::string s;
        char buf[4096];
        size_t got;
        while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, got);
        std::fclose(f);
        size_t pos = 0;
        for (;;) {
            const size_t k = s.find("\"key\"", pos);
            if (k == std::string::npos) break;
            const size_t q0 = s.find('"', s.find(':', k) + 1);
            const size_t q1 = q0 == std::string::npos ? q0 : s.find('"', q0 + 1);
            if (q1 == std::string::npos) break;
            const size_t end = s.find('}', q1);
            Entry E;
            E.key = s.substr(q0 + 1, q1 - q0 - 1);
            sbt_batch_tuning_default(&E.t);
            const double split = field(s, q1, end, "split_n");
            const double tail = field(s, q1, end, "tail_words");
            const double fill = field(s, q1, end, "fill");
            pos = end == std::string::npos ? s.size() : end;
            if (!std::isfinite(split) || !std::isfinite(tail) || !std::isfinite(fill)) continue;
            E.t.split_n = static_cast<int32_t>(split);
            E.t.tail_words = static_cast<int32_t>(tail);
            E.t.fill = fill;
            const double band = field(s, q1, end, "band_rows");
            E.t.band_rows = std::isfinite(band) ? static_cast<int32_t>(band) : 0;
            E.t.from_cache = 1;
            const size_t h = E.key.find(" h=");
            if (h == std::string::npos) continue;
            E.prefix = E.key.substr(0, h);
            std::vector<double> hist;
            double tot = 0.0;
            for (const char *c = E.key.c_str() + h + 3; *c;) {
                char *next = nullptr;
                const double v = std::strtod(c, &next);
                if (next == c) break;
                hist.push_back(v);
                tot += v;
                c = *next == ',' ? next + 1 : next;
            }
            if (static_cast<int>(hist.size()) != kBuckets || !(tot > 0)) continue;
            for (double &v : hist) v /= tot;
            E.hist = hist;
            all.push_back(E);
        }
    });
    return all;
}

}  // namespace

extern "C" int sbt_batch_tuning_key(const int32_t *n, int32_t n_events, sbt_mode mode,
                                    sbt_precision prec, int32_t agents, char *key, size_t key_len) {
    const char *who = "sbt_batch_tuning_key";
    sbt::clear_error();
    if (!n || n_events < 1 || !key || key_len == 0 || agents < 1)
        return sbt::fail(SBT_EINVAL, "%s: invalid argument", who);
    if (mode != SBT_BSB && mode != SBT_DSB && mode != SBT_ASB)
        return sbt::fail(SBT_EINVAL, "%s: unknown mode", who);
    if (prec != SBT_PREC_FP16 && prec != SBT_PREC_BF16)
        return sbt::fail(SBT_EUNSUPPORTED, "%s: batches hold FP16 or BF16 couplings", who);
    const std::string k = key_of(prefix_of(mode, prec, agents), histogram(n, n_events));
    if (k.size() + 1 > key_len) return sbt::fail(SBT_EINVAL, "%s: key buffer too short", who);
    std::memcpy(key, k.c_str(), k.size() + 1);
    return SBT_OK;
}

extern "C" int sbt_batch_tuning_lookup(const int32_t *n, int32_t n_events, sbt_mode mode,
                                       sbt_precision prec, int32_t agents, sbt_batch_tuning *out) {
    const char *who = "sbt_batch_tuning_lookup";
    if (!out) {
        sbt::clear_error();
        return sbt::fail(SBT_EINVAL, "%s: out is NULL", who);
    }
    char key[256];
    const int rc = sbt_batch_tuning_key(n, n_events, mode, prec, agents, key, sizeof key);
    if (rc) return rc;
    sbt_batch_tuning_default(out);
    const std::string prefix = prefix_of(mode, prec, agents);
    const std::vector<int64_t> h = histogram(n, n_events);
    std::vector<double> hn(kBuckets);
    for (int i = 0; i < kBuckets; ++i) hn[i] = static_cast<double>(h[i]) / n_events;
    const Entry *best = nullptr;
    double best_d = 0.25;
    for (const Entry &E : entries()) {
        if (E.key == key) {
            best = &E;
            break;
        }
        if (E.prefix != prefix) continue;
        double d = 0.0;
        for (int i = 0; i < kBuckets; ++i) d += std::fabs(E.hist[i] - hn[i]);
        if (d <= best_d) {
            best_d = d;
            best = &E;
        }
    }
    if (best) *out = best->t;
    return SBT_OK;
}
