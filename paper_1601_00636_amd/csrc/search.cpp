// Resumable background search over region (1.2), after the search loop of
// section 5: a host thread scans row after row from a starting (p, q), in
// chunks of whole hundreds of p sized to a few tens of milliseconds of GPU
// work, and keeps the exit point, the deepest prime used in the last hundred
// of p (r_max), running totals and the pairs that passed every prime.  A stop
// takes effect at the next row boundary and appends the paper's report line
// (time stamp, exit p and q, r_max) to the report file; a new search started
// from that exit point continues exactly where the old one stopped.
#include <string.h>
#include <time.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <mutex>
#include <string>
#include <thread>

#include "runtime.h"

using namespace cuboid;

namespace {

constexpr uint32_t kSearchMinP = 152;           // (5.2) holds from p = 152 on
constexpr uint64_t kChunkPairs = 250000000000ull;   // some 15-50 ms of sweep
constexpr uint64_t kChunkMaxRows = 1u << 20;
constexpr uint64_t kKeepSurvivors = 1u << 20;
constexpr uint64_t kChunkSurvCap = 1u << 16;

uint32_t least_q(uint32_t p) {
    uint32_t a = 1;
    while (9ull * a * a * a < p) ++a;
    const uint32_t lin = (uint32_t)(((uint64_t)p + 58) / 59);
    return std::min(a, lin);
}

}  // namespace

struct cuboid_search {
    cuboid_ctx *ctx = nullptr;
    std::vector<uint32_t> primes;
    uint32_t r_last = 0;          // largest prime of the list
    uint32_t p_end = 0;
    std::string report_path;
    std::thread th;
    std::atomic<bool> stop{false};
    std::mutex mu;                // guards everything below
    cuboid_search_report rep;
    std::vector<uint64_t> surv;   // p * 2^32 + q, ascending, the first kKeepSurvivors
    uint32_t hundred = 0;         // hundred of p that rep.r_max belongs to
};

namespace {

// deepest prime used by a set of pairs, from its first-rejecter counts
uint32_t depth_of(const uint32_t *primes, const uint64_t *counts, uint32_t n, uint64_t pairs,
                  uint64_t survivors, uint32_t r_last) {
    if (pairs == 0) return 1;
    if (survivors) return r_last;
    uint32_t d = 1;
    for (uint32_t i = 0; i < n; ++i)
        if (counts[i]) d = std::max(d, primes[i]);
    return d;
}

void note_depth(cuboid_search *s, uint32_t p, uint32_t d) {
    // r_max starts again at 1 for each hundred of p
    if (p / 100 != s->hundred) {
        s->hundred = p / 100;
        s->rep.r_max = 1;
    }
    s->rep.r_max = std::max(s->rep.r_max, d);
}

void finish(cuboid_search *s, int status) {
    std::lock_guard<std::mutex> g(s->mu);
    s->rep.status = status;
    s->rep.running = 0;
    s->rep.unix_time = (int64_t)time(nullptr);
}

// One step: the rest of a started row, or whole rows up to a hundred boundary.
int step(cuboid_search *s, uint32_t p, uint32_t q, uint32_t *p_next) {
    cuboid_ctx *ctx = s->ctx;
    const uint32_t n = (uint32_t)s->primes.size();
    std::vector<uint64_t> counts(n, 0), surv;
    uint64_t pairs = 0, nsurv = 0;
    // callers waiting for the context go first
    while (ctx->waiting.load() > 0) std::this_thread::sleep_for(std::chrono::microseconds(50));
    std::lock_guard<std::recursive_mutex> g(ctx->mu);
    if (hipSetDevice(ctx->device) != hipSuccess) return CUBOID_E_DEVICE;
    if (q > least_q(p)) {
        // the rest of row p from column q
        cuboid_request rect;
        rect.p0 = rect.p1 = p;
        rect.q0 = q;
        rect.q1 = 59u * p;
        SieveOut &so = ctx->h_out;
        int st = sieve_rects(ctx, s->primes, &rect, 1, kChunkSurvCap, ctx->stream, &so);
        if (st && st != CUBOID_E_LIMIT) return st;
        memcpy(counts.data(), so.counts, (size_t)n * 8);
        pairs = so.pairs[0];
        nsurv = so.n_surv;
        for (const SurvEntry &e : so.surv) surv.push_back(((uint64_t)p << 32) | (q + e.idx));
        std::lock_guard<std::mutex> gs(s->mu);
        note_depth(s, p, depth_of(s->primes.data(), counts.data(), n, pairs, nsurv, s->r_last));
        *p_next = p + 1;
    } else {
        // whole rows: the rest of this hundred, or whole hundreds
        // about 0.6 * 59 p' coprime pairs in row p': R rows from p hold about
        // 36 (p R + R^2 / 2); solve for the chunk's pair budget
        const double pd = (double)p;
        uint64_t rows = (uint64_t)(std::sqrt(pd * pd + 2.0 * (double)kChunkPairs / 36.0) - pd);
        rows = std::max<uint64_t>(1, std::min(rows, kChunkMaxRows));
        uint64_t end;
        if (p % 100) end = (p / 100 + 1) * 100ull - 1;
        else end = p + std::max<uint64_t>(100, rows / 100 * 100) - 1;
        end = std::min<uint64_t>(end, s->p_end);
        const uint32_t pb = (uint32_t)end;
        const uint64_t n_bands = (pb - p) / 100 + 1;
        std::vector<uint32_t> r_max(n_bands, 1);
        surv.resize(kChunkSurvCap);
        int st = region_sieve(ctx, p, pb, 100, s->primes, surv.data(), surv.size(), &nsurv,
                              counts.data(), &pairs, r_max.data(), ctx->stream);
        if (st && st != CUBOID_E_CAPACITY) return st;
        surv.resize(std::min<uint64_t>(nsurv, surv.size()));
        std::lock_guard<std::mutex> gs(s->mu);
        for (uint64_t b = 0; b < n_bands; ++b) note_depth(s, (uint32_t)(p + 100 * b), r_max[b]);
        *p_next = pb + 1;
    }
    std::lock_guard<std::mutex> gs(s->mu);
    s->rep.pairs += pairs;
    s->rep.survivors += nsurv;
    for (uint64_t v : surv)
        if (s->surv.size() < kKeepSurvivors) s->surv.push_back(v);
    return CUBOID_OK;
}

void worker(cuboid_search *s, uint32_t p, uint32_t q) {
    while (!s->stop.load()) {
        uint32_t p_next = p;
        const int st = step(s, p, q, &p_next);
        if (st) { finish(s, st); return; }
        p = p_next;
        if (p > s->p_end) break;
        q = least_q(p);   // every later row is scanned from its least q
        {
            std::lock_guard<std::mutex> g(s->mu);
            s->rep.p = p;
            s->rep.q = p <= kRegionMaxP ? least_q(p) : 0;
            s->rep.p_hundred = p / 100 * 100;
        }
    }
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->rep.p = p;
        s->rep.q = p <= kRegionMaxP ? least_q(p) : 0;
        s->rep.p_hundred = p / 100 * 100;
    }
    finish(s, CUBOID_OK);
}

void write_report(const cuboid_search *s, const cuboid_search_report &r) {
    if (s->report_path.empty()) return;
    FILE *f = fopen(s->report_path.c_str(), "a");
    if (!f) return;
    const time_t t = (time_t)r.unix_time;
    struct tm tmv;
    localtime_r(&t, &tmv);
    fprintf(f, "%d-%d-%d %02d:%02d\nStop with p=%u, q=%u, r_max=%u\n", tmv.tm_year + 1900,
            tmv.tm_mon + 1, tmv.tm_mday, tmv.tm_hour, tmv.tm_min, r.p, r.q, r.r_max);
    fclose(f);
}

}  // namespace

extern "C" {

int cuboid_search_start(cuboid_ctx *ctx, const uint32_t *primes, uint32_t n_primes, uint32_t p,
                        uint32_t q, uint32_t p_end, const char *report_path,
                        cuboid_search **out) {
    if (!out) return CUBOID_E_ARG;
    *out = nullptr;
    CTX_ENTER(ctx);
    if (p < kSearchMinP) return CUBOID_E_RANGE;
    if (p > kRegionMaxP) return CUBOID_E_LIMIT;
    if (q < least_q(p) || q > 59u * p) return CUBOID_E_RANGE;
    if (p_end == 0 || p_end > kRegionMaxP) p_end = kRegionMaxP;
    if (p_end < p) return CUBOID_E_RANGE;
    std::vector<uint32_t> sorted;
    int st = canonical_primes(primes, n_primes, &sorted);
    if (st) return st;
    int expected = 0;
    if (!ctx->searches.compare_exchange_strong(expected, 1)) return CUBOID_E_BUSY;
    cuboid_search *s = new cuboid_search();
    s->ctx = ctx;
    s->primes.assign(primes, primes + n_primes);
    s->r_last = sorted.back();
    s->p_end = p_end;
    if (report_path) s->report_path = report_path;
    memset(&s->rep, 0, sizeof(s->rep));
    s->rep.p = p;
    s->rep.q = q;
    s->rep.p_hundred = p / 100 * 100;
    s->rep.r_max = 1;
    s->rep.running = 1;
    s->rep.unix_time = (int64_t)time(nullptr);
    s->hundred = p / 100;
    s->th = std::thread(worker, s, p, q);
    *out = s;
    return CUBOID_OK;
}

int cuboid_search_current(cuboid_search *s, cuboid_search_report *out) {
    if (!s || !out) return CUBOID_E_ARG;
    std::lock_guard<std::mutex> g(s->mu);
    *out = s->rep;
    if (s->rep.running) out->unix_time = (int64_t)time(nullptr);
    return CUBOID_OK;
}

int cuboid_search_survivors(cuboid_search *s, uint64_t *pq, uint64_t cap, uint64_t *n) {
    if (!s || !n || (cap && !pq)) return CUBOID_E_ARG;
    std::lock_guard<std::mutex> g(s->mu);
    *n = s->surv.size();
    const uint64_t k = std::min<uint64_t>(cap, s->surv.size());
    if (k) memcpy(pq, s->surv.data(), k * 8);
    return s->surv.size() > cap ? CUBOID_E_CAPACITY : CUBOID_OK;
}

int cuboid_search_stop(cuboid_search *s, cuboid_search_report *out) {
    if (!s) return CUBOID_E_ARG;
    s->stop.store(true);
    if (s->th.joinable()) s->th.join();
    cuboid_search_report r;
    {
        std::lock_guard<std::mutex> g(s->mu);
        r = s->rep;
    }
    r.unix_time = (int64_t)time(nullptr);
    write_report(s, r);
    if (out) *out = r;
    s->ctx->searches.store(0);
    delete s;
    return r.status;
}

}  // extern "C"
