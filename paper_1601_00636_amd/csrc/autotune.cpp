// Autotuner: times the sweep for candidate tunings (number of dense primes K
// and persistent grid size, then for the best of those the work sharing:
// schedule and piece size) on a sample and keeps the fastest for the prime
// set.  Choices are cached as JSON lines keyed by device architecture
// and prime set.  Results never depend on the tuning (the dense primes are an
// ascending prefix and every count is the first rejecting prime).
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>

#include "runtime.h"

using namespace cuboid;

namespace {

std::string prime_key(const std::vector<uint32_t> &primes) {
    // FNV-1a over the sorted list, plus its length and ends for readability
    uint64_t h = 1469598103934665603ull;
    for (uint32_t r : primes) {
        for (int b = 0; b < 4; ++b) {
            h ^= (r >> (8 * b)) & 0xff;
            h *= 1099511628211ull;
        }
    }
    char buf[96];
    snprintf(buf, sizeof(buf), "n%zu_%u_%u_%016llx", primes.size(), primes.front(), primes.back(),
             (unsigned long long)h);
    return buf;
}

bool read_cache(const char *path, const std::string &arch, const std::string &key,
                cuboid_tuning *out) {
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (fgets(line, sizeof(line), f)) {
        if (!strstr(line, ("\"arch\": \"" + arch + "\"").c_str())) continue;
        if (!strstr(line, ("\"primes\": \"" + key + "\"").c_str())) continue;
        unsigned k = 0, w = 0, b = 0;
        const char *pk = strstr(line, "\"dense_primes\": ");
        const char *pw = strstr(line, "\"workgroups\": ");
        const char *pb = strstr(line, "\"lds_budget\": ");
        if (!pk || !pw || !pb) continue;
        if (sscanf(pk, "\"dense_primes\": %u", &k) != 1) continue;
        if (sscanf(pw, "\"workgroups\": %u", &w) != 1) continue;
        if (sscanf(pb, "\"lds_budget\": %u", &b) != 1) continue;
        unsigned sc = 0, pc = 0;   // absent from older lines: the defaults
        const char *ps = strstr(line, "\"schedule\": ");
        const char *pp = strstr(line, "\"piece_units\": ");
        if (ps && sscanf(ps, "\"schedule\": %u", &sc) != 1) continue;
        if (pp && sscanf(pp, "\"piece_units\": %u", &pc) != 1) continue;
        if (sc > 3 || pc > (1u << 20)) continue;
        out->dense_primes = k;
        out->workgroups = w;
        out->lds_budget = b;
        out->schedule = sc;
        out->piece_units = pc;
        found = true;   // the last matching line wins
    }
    fclose(f);
    return found;
}

void append_cache(const char *path, const std::string &arch, const std::string &key,
                  const cuboid_tuning &t, double ms) {
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f,
            "{\"arch\": \"%s\", \"primes\": \"%s\", \"dense_primes\": %u, \"workgroups\": %u, "
            "\"lds_budget\": %u, \"schedule\": %u, \"piece_units\": %u, \"sample_ms\": %.4f}\n",
            arch.c_str(), key.c_str(), t.dense_primes, t.workgroups, t.lds_budget, t.schedule,
            t.piece_units, ms);
    fclose(f);
}

// Times every candidate on the sample and keeps the fastest.  A sample that
// overflows the survivor scratch still times the whole sweep, so E_LIMIT and
// E_CAPACITY count as a completed run.
int tune(cuboid_ctx *ctx, const std::vector<uint32_t> &sorted, const cuboid_request *sample,
         uint32_t n_sample, const std::string &key, const char *cache_path, cuboid_tuning *out) {
    const std::string arch(ctx->arch);
    cuboid_tuning best;
    if (cache_path && read_cache(cache_path, arch, key, &best)) {
        ctx->tunings[sorted] = best;
        if (out) *out = best;
        return CUBOID_OK;
    }
    Plan *pl = nullptr;
    int st = build_plan(ctx, sorted, &pl);
    if (st) return st;
    const uint32_t budget = (uint32_t)(ctx->max_lds - kSweepFixedLds);   // dense tables: all the LDS left
    const uint32_t kmax = default_dense(*pl, budget);
    const uint32_t cus = (uint32_t)ctx->cu_count;
    const bool saved_timing = ctx->timing;
    ctx->timing = true;
    double best_ms = 1e30;
    best.dense_primes = 0; best.workgroups = cus; best.lds_budget = budget; best.schedule = 0;
    best.piece_units = 0;
    // the median sweep time of five runs under tuning t (a best-of-few
    // would favour tunings whose time varies most from run to run)
    auto time_of = [&](const cuboid_tuning &t, double *ms) -> int {
        ctx->tunings[sorted] = t;
        double v[5];
        for (int rep = 0; rep < 5; ++rep) {
            int r = sieve_rects(ctx, sorted, sample, n_sample, 1 << 16, ctx->stream, &ctx->h_out);
            if (r == CUBOID_E_LIMIT || r == CUBOID_E_CAPACITY) r = CUBOID_OK;
            if (r) return r;
            v[rep] = ctx->last.sweep_ms;
        }
        std::sort(v, v + 5);
        *ms = v[2];
        return CUBOID_OK;
    };
    const uint32_t klo = kmax > 5 ? kmax - 5 : 0;
    // one workgroup fills a compute unit's LDS, so grids beyond the CU count
    // run as successive waves of workgroups: smaller pieces that even out
    // the finishing times of unequal units
    const uint32_t wgs[4] = {cus, 2 * cus, 4 * cus, 8 * cus};
    for (uint32_t K = klo; K <= kmax && !st; ++K) {
        for (uint32_t w : wgs) {
            cuboid_tuning t;
            t.dense_primes = K; t.workgroups = w; t.lds_budget = budget; t.schedule = 0;
            t.piece_units = 0;
            double ms = 0;
            st = time_of(t, &ms);
            if (st) break;
            if (ms < best_ms) { best_ms = ms; best = t; }
        }
    }
    // the work sharing for the best K and grid: workgroup pieces of fixed
    // sizes, round-robin pieces per wave, the shared counter
    const uint32_t shares[8][2] = {{0, 64}, {0, 128}, {0, 512}, {0, 1024},
                                   {0, 4096}, {1, 0}, {1, 64}, {2, 0}};
    const cuboid_tuning base = best;
    for (int i = 0; i < 8 && !st; ++i) {
        cuboid_tuning t = base;
        t.schedule = shares[i][0];
        t.piece_units = shares[i][1];
        double ms = 0;
        st = time_of(t, &ms);
        if (!st && ms < best_ms) { best_ms = ms; best = t; }
    }
    ctx->timing = saved_timing;
    if (st) {
        ctx->tunings.erase(sorted);
        return st;
    }
    ctx->tunings[sorted] = best;
    if (cache_path) append_cache(cache_path, arch, key, best, best_ms);
    if (out) *out = best;
    return CUBOID_OK;
}

uint64_t sample_hash(const cuboid_request *r, uint32_t n) {
    uint64_t h = 1469598103934665603ull;
    for (uint32_t i = 0; i < n; ++i) {
        const uint32_t v[4] = {r[i].p0, r[i].p1, r[i].q0, r[i].q1};
        for (uint32_t x : v)
            for (int b = 0; b < 4; ++b) {
                h ^= (x >> (8 * b)) & 0xff;
                h *= 1099511628211ull;
            }
    }
    return h;
}

}  // namespace

extern "C" int cuboid_autotune(cuboid_ctx *ctx, const uint32_t *primes, uint32_t n_primes,
                               const char *cache_path, cuboid_tuning *out) {
    CTX_ENTER(ctx);
    std::vector<uint32_t> sorted;
    int st = canonical_primes(primes, n_primes, &sorted);
    if (st) return st;
    CtxLock g(ctx);
    if (hipSetDevice(ctx->device) != hipSuccess) return CUBOID_E_DEVICE;
    // sample: 32768 rows x 65536 columns near 2^19 (the scale of the batched
    // workloads), about 2^19 units: enough work per wave for the timing to
    // reflect a full launch
    cuboid_request rect;
    rect.p0 = 1u << 19; rect.p1 = (1u << 19) + 32767;
    rect.q0 = 1u << 19; rect.q1 = (1u << 19) + 65535;
    return tune(ctx, sorted, &rect, 1, prime_key(sorted), cache_path, out);
}

extern "C" int cuboid_autotune_for(cuboid_ctx *ctx, const uint32_t *primes, uint32_t n_primes,
                                   const cuboid_request *sample, uint32_t n_sample,
                                   const char *cache_path, cuboid_tuning *out) {
    CTX_ENTER(ctx);
    if (!sample || n_sample == 0 || n_sample == 0xffffffffu) return CUBOID_E_ARG;
    for (uint32_t i = 0; i < n_sample; ++i)
        if (rect_valid(sample[i].p0, sample[i].p1, sample[i].q0, sample[i].q1))
            return CUBOID_E_RANGE;
    std::vector<uint32_t> sorted;
    int st = canonical_primes(primes, n_primes, &sorted);
    if (st) return st;
    CtxLock g(ctx);
    if (hipSetDevice(ctx->device) != hipSuccess) return CUBOID_E_DEVICE;
    char w[40];
    snprintf(w, sizeof(w), "_w%u_%016llx", n_sample,
             (unsigned long long)sample_hash(sample, n_sample));
    return tune(ctx, sorted, sample, n_sample, prime_key(sorted) + w, cache_path, out);
}
