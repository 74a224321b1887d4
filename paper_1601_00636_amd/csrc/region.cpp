// The sieve over region (1.2) of Theorem 1.2, as scanned in sections 5 and 6:
// for every p in [p0, p1] every q with min(cbrt(p / 9), p / 59) <= q <= 59 p,
// in the domain of Conjecture 1.1 (coprime, p != q).
//
// Rows are grouped into report bands of `band_rows` consecutive p (the
// paper's progress report uses hundreds), one counter slot per band, so the
// deepest prime used in each band comes out of its first-rejecter counts.
// Rows go to the sweep as sub-requests whose column range is
// [qmin(first row), 59 * last row]; each lane then keeps only its own row's
// columns.  Sub-requests hold about p / 64 rows, so the spread of 59 p over a
// sub-request stays near 1/64 of a row's length.  With bands of 64 rows or
// more, sub-requests run across band edges and every lane counts into its own
// row's band, so no lane idles at a band's last, partial block of 64 rows;
// narrower bands get sub-requests of their own.
#include <string.h>

#include <algorithm>

#include "runtime.h"

namespace cuboid {

namespace {

constexpr uint32_t kSlotsPerCall = 1u << 15;   // report bands per sweep
constexpr uint64_t kSubMinRows = 64, kSubMaxRows = 8192;

// least a >= 1 with 9 a^3 >= p, by bisection on [1, 256]
uint32_t cube_bound(uint32_t p) {
    uint32_t lo = 1, hi = 256;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) / 2;
        if (9ull * mid * mid * mid >= p) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

uint32_t region_qmin_host(uint32_t p) {
    const uint32_t lin = (uint32_t)(((uint64_t)p + 58) / 59);
    return std::min(cube_bound(p), lin);
}

uint64_t sub_rows(uint64_t p) {
    uint64_t b = (p >> 12) << 6;
    return std::max(kSubMinRows, std::min(kSubMaxRows, b));
}

}  // namespace

int region_sieve(cuboid_ctx *ctx, uint32_t p0, uint32_t p1, uint32_t band_rows,
                 const std::vector<uint32_t> &caller_primes, uint64_t *survivors, uint64_t cap,
                 uint64_t *n_survivors, uint64_t *counts, uint64_t *n_pairs, uint32_t *r_max,
                 hipStream_t s) {
    Plan *pl = nullptr;
    DenseSet *ds = nullptr;
    cuboid_tuning tun;
    int st = prepare_primes(ctx, caller_primes, &pl, &tun, &ds);
    if (st) return st;
    const uint32_t np = (uint32_t)caller_primes.size();
    const std::vector<int32_t> col = count_columns(*pl, caller_primes);
    const uint64_t rows = (uint64_t)p1 - p0 + 1;
    const uint64_t n_bands = (rows + band_rows - 1) / band_rows;
    const uint64_t surv_cap = std::min<uint64_t>(cap, kMaxSurvScratch);
    const uint32_t r_last = pl->primes.back();

    std::vector<uint64_t> total(np, 0);
    uint64_t pairs = 0, found = 0;
    CoreOut sum;
    if (ctx->timing && hipEventRecord(ctx->ev_total0, s) != hipSuccess) return CUBOID_E_DEVICE;
    for (uint64_t b0 = 0; b0 < n_bands; b0 += kSlotsPerCall) {
        const uint32_t nb = (uint32_t)std::min<uint64_t>(kSlotsPerCall, n_bands - b0);
        std::vector<ReqDesc> &reqs = ctx->h_reqs;
        reqs.clear();
        if (band_rows >= (uint32_t)kWave) {
            // sub-requests run across band edges; each lane counts into the
            // slot of its own row's band (a 64-row block meets two at most)
            const uint64_t first = p0 + b0 * band_rows;
            const uint64_t last = std::min<uint64_t>(p1, first + (uint64_t)nb * band_rows - 1);
            for (uint64_t a = first; a <= last;) {
                const uint64_t e = std::min<uint64_t>(last, a + sub_rows(a) - 1);
                const uint32_t j = (uint32_t)((a - first) / band_rows);
                ReqDesc d;
                memset(&d, 0, sizeof(d));
                d.p0 = (uint32_t)a;
                d.p1 = (uint32_t)e;
                d.q0 = region_qmin_host((uint32_t)a);
                d.q1 = 59u * (uint32_t)e;
                d.ip0 = (uint32_t)a;
                d.slot = j;
                d.flags = kReqRegion | kReqBandSplit;
                d.band_rows = band_rows;
                d.band_p0 = (uint32_t)(first + (uint64_t)j * band_rows);
                reqs.push_back(d);
                a = e + 1;
            }
        }
        for (uint32_t j = 0; j < nb && band_rows < (uint32_t)kWave; ++j) {
            const uint64_t ba = p0 + (b0 + j) * band_rows;
            const uint64_t bb = std::min<uint64_t>(p1, ba + band_rows - 1);
            for (uint64_t a = ba; a <= bb;) {
                const uint64_t e = std::min<uint64_t>(bb, a + sub_rows(a) - 1);
                ReqDesc d;
                memset(&d, 0, sizeof(d));
                d.p0 = (uint32_t)a;
                d.p1 = (uint32_t)e;
                d.q0 = region_qmin_host((uint32_t)a);
                d.q1 = 59u * (uint32_t)e;
                d.ip0 = (uint32_t)a;
                d.slot = j;
                d.flags = kReqRegion;
                reqs.push_back(d);
                a = e + 1;
            }
        }
        CoreOut &co = ctx->h_core;
        st = sieve_core(ctx, *pl, *ds, tun, reqs, nb, nullptr, surv_cap, s, &co);
        if (st) return st;
        sum.units += co.units;
        sum.sweep_ms += co.sweep_ms;
        for (uint32_t j = 0; j < nb; ++j) {
            const uint64_t *c = co.counts + (size_t)j * co.width;
            uint64_t rejected = 0;
            uint32_t deepest = 0;
            for (uint32_t k = 0; k < co.nc; ++k) {
                rejected += c[k];
                if (c[k]) deepest = pl->primes[pl->nontriv_idx[k]];
            }
            for (uint32_t i = 0; i < np; ++i)
                if (col[i] >= 0) total[i] += c[col[i]];
            pairs += co.pairs[j];
            // the largest prime some pair of the band was tested against:
            // its deepest first rejecter, or the whole list if a pair survived
            if (r_max) r_max[b0 + j] = co.pairs[j] == 0 ? 1 : (co.pairs[j] > rejected ? r_last : deepest);
        }
        if (co.n_surv > surv_cap && cap > surv_cap) return CUBOID_E_LIMIT;
        for (const SurvEntry &e : co.surv)
            if (found < cap) survivors[found++] = e.idx;
            else ++found;
        if (co.n_surv > co.surv.size()) found += co.n_surv - co.surv.size();
    }
    memcpy(counts, total.data(), (size_t)np * 8);
    *n_pairs = pairs;
    *n_survivors = found;
    record_timing(ctx, s, sum, *ds, tun);
    return found > cap ? CUBOID_E_CAPACITY : CUBOID_OK;
}

}  // namespace cuboid
