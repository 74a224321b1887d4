// The sieve sweep of arXiv:1601.00636, section 2, on CDNA4.
//
// Each wavefront owns 64 rows p (one per lane; the rows of a request, taken in
// an order that groups them by number of prime factors) and walks the columns
// q in windows of 64, so one 64-bit mask per lane holds the state of 64 pairs.
// Per window:
//   1. coprimality (Conjecture 1.1 domain): a wheel lookup gives the q sharing
//      no factor 2, 3 or 5 with p, and each prime factor >= 7 of p clears its
//      multiples by a shifted bit pattern;
//   2. dense primes: for the first K non-trivial primes r (ascending) one LDS
//      read fetches u_r(p mod r, q mod r) for all 64 columns at once, the
//      pairs it rejects are counted for r and dropped;
//   3. the rare windows with pairs left are queued per wave; when 64 are
//      queued every lane takes one and tests its pairs against the remaining
//      primes in ascending order through the ratio-form tables, so the first
//      rejecting prime is counted and unrejected pairs are appended as
//      survivors.
// The flattened space of 64x64 units over all requests of a launch is shared
// by the waves of a persistent grid: pieces dealt round-robin to the
// workgroups and taken by their waves through an LDS cursor (the default), or
// round-robin pieces per wave, or a shared counter in global memory (see the
// work-sharing comment in the kernel).
#include "devmath.h"
#include "internal.h"

namespace cuboid {

namespace {

struct QEntry {
    uint32_t p;
    uint32_t qb;
    uint64_t mask;
};
static_assert(sizeof(QEntry) == kQueueEntryBytes, "queue entry size");

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
    return ((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v);
}

// Sum over the wave with DPP moves (no LDS round trips): an inclusive scan
// within each row of 16 lanes (row_shr 1, 2, 4, 8), then lane 15 of rows 0 and
// 2 added into rows 1 and 3 (row_bcast:15) and lane 31 into rows 2 and 3
// (row_bcast:31); lane 63 ends with the total.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
    int x = (int)v;
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return (uint32_t)__builtin_amdgcn_readlane(x, 63);
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t w = __shfl_xor(v, o, kWave);
        v = w > v ? w : v;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t w = __shfl_xor(v, o, kWave);
        v = w < v ? w : v;
    }
    return v;
}

__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Least q >= 1 that region (1.2) allows in row p >= 1: the smaller of the
// least a with 9 a^3 >= p and of ceil(p / 59).  a <= 256 covers every
// p <= 9 * 256^3, beyond the largest row a region may hold.
__device__ __forceinline__ uint32_t region_qmin(uint32_t p) {
    uint32_t lo = 1, hi = 256;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (9ull * mid * mid * mid >= p) hi = mid; else lo = mid + 1;
    }
    const uint32_t b = p / 59 + (p % 59 != 0);
    return lo < b ? lo : b;
}

// x mod d for a per-lane divisor d >= 1 (used at segment setup only)
__device__ __forceinline__ uint32_t mod_var(uint32_t x, uint32_t d) { return x % d; }

// entry offset of the multiple patterns of a prime l in 7..61 (others unused)
__constant__ uint16_t c_pat_off[64] = {
    0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 7, 0, 18, 0, 0, 0, 31, 0, 48, 0, 0, 0, 67, 0, 0, 0, 0, 0, 90,
    0, 119, 0, 0, 0, 0, 0, 150, 0, 0, 0, 187, 0, 228, 0, 0, 0, 271, 0, 0, 0, 0, 0, 318, 0, 0, 0, 0,
    0, 371, 0, 430, 0, 0};

// Tests the pairs of one queued window against the deep primes, in ascending
// order; counts the first rejecting prime, appends unrejected pairs.  Counts
// of the wave's current slot `slot0` go to its LDS counters, counts of another
// slot (the second band of a band-split row block) straight to global memory.
template <bool SPLIT>
__device__ __forceinline__ void deep_window(const SweepParams &P, const QEntry e,
                                            const ReqDesc &R, uint32_t slot0, uint32_t *dcnt,
                                            unsigned long long *cnt_rep) {
    const uint32_t slot = (SPLIT && (R.flags & kReqBandSplit))
                              ? R.slot + (e.p - R.band_p0) / R.band_rows
                              : R.slot;
    uint64_t mask = e.mask;
    const uint64_t width = (uint64_t)R.q1 - R.q0 + 1;
    while (mask) {
        const uint32_t j = __builtin_ctzll(mask);
        mask &= mask - 1;
        const uint32_t q = e.qb + j;
        bool rejected = false;
        for (uint32_t i = 0; i < P.n_deep; ++i) {
            const DeepPrime d = P.deep[i];
            const uint32_t a = modr(e.p, d.r, d.m), b = modr(q, d.r, d.m);
            if (a == 0 || b == 0) continue;
            const uint32_t x = mulr(a, P.ipool[d.ioff + b], d.r, d.m);
            if (P.vpool[d.voff + x]) {
                if (i < kDeepCounters && (!SPLIT || slot == slot0))
                    atomicAdd(&dcnt[i], 1u);
                else
                    atomicAdd(&cnt_rep[(uint64_t)slot * P.nc + P.K + i], 1ull);
                rejected = true;
                break;
            }
        }
        if (!rejected) {
            const unsigned long long pos = atomicAdd(P.surv_n, 1ull);
            if (pos < P.surv_cap) {
                SurvEntry s;
                s.idx = (R.flags & kReqRegion) ? ((uint64_t)e.p << 32) | q
                                               : (uint64_t)(e.p - R.ip0) * width + (q - R.q0);
                s.req = slot;
                s.pad = 0;
                P.surv[pos] = s;
            }
        }
    }
}

__device__ __forceinline__ uint64_t lds64(const unsigned char *base, uint32_t byte_off) {
    return *(const uint64_t *)(base + byte_off);
}

constexpr uint32_t kFlushWindows = 1u << 19;   // per-lane u32 counters stay below 2^31
constexpr uint64_t kMinClaim = 16;             // smallest claim from a cursor or counter
constexpr uint64_t kPiece = 256;               // largest round-robin piece
constexpr uint64_t kBigPiece = 4096;           // workgroup pieces of launches with many units
constexpr uint64_t kWgPieces = 32;             // workgroup pieces per workgroup, at least

// KD dense primes; MF factor slots (enough for every row of the launch);
// SPLIT: the launch holds band-split region requests
template <int KD, int MF, bool SPLIT>
__global__ void __launch_bounds__(kWave * kWavesPerWG) sweep_kernel(const SweepParams P) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid >> 6;
    // LDS: dense window tables | wheel | multiple patterns | per-wave queue + counters
    uint64_t *sdense = (uint64_t *)smem;
    uint64_t *swheel = sdense + P.dense_words;
    uint64_t *spat = swheel + kWheelSubsets * kWheel;
    unsigned char *wave_area = (unsigned char *)(spat + kPatEntries) + (size_t)wv * kPerWaveBytes;
    QEntry *queue = (QEntry *)wave_area;
    uint32_t *dcnt = (uint32_t *)(wave_area + kQueueCap * sizeof(QEntry));
    unsigned long long *wg_cursor =
        (unsigned long long *)((unsigned char *)(spat + kPatEntries) + kWavesPerWG * kPerWaveBytes);

    for (uint32_t i = tid; i < P.dense_words; i += blockDim.x) sdense[i] = P.dense_tab[i];
    for (uint32_t i = tid; i < kWheelSubsets * kWheel; i += blockDim.x) swheel[i] = P.wheel[i];
    for (uint32_t i = tid; i < (uint32_t)kPatEntries; i += blockDim.x) spat[i] = P.patterns[i];
    for (uint32_t i = lane; i < kDeepCounters; i += kWave) dcnt[i] = 0;
    if (tid == 0) *wg_cursor = 0;
    __syncthreads();

    const uint32_t wheel_byte = P.dense_words * 8;
    const uint32_t pat_byte = wheel_byte + kWheelSubsets * kWheel * 8;
    const uint64_t nwaves = (uint64_t)gridDim.x * kWavesPerWG;
    const uint64_t w = (uint64_t)blockIdx.x * kWavesPerWG + wv;
    const uint64_t n_units = P.units_dev ? uni64(*P.units_dev) : P.n_units;
    const uint32_t rep = uni((uint32_t)(w & (P.n_rep - 1)));
    unsigned long long *cnt_rep = P.counts + (uint64_t)rep * P.rep_stride_counts;
    unsigned long long *pairs_rep = P.pairs + (uint64_t)rep * P.rep_stride_pairs;
    uint32_t ri = 0;   // request holding the current unit

    // per lane: coprime pairs seen, and pairs left after each dense prime (the
    // two 32-bit halves of a window's mask counted separately, so that each
    // popcount accumulates in one instruction)
    uint32_t left[KD + 1], left_hi[KD + 1];
    for (int k = 0; k <= KD; ++k) { left[k] = 0; left_hi[k] = 0; }
    uint32_t npairs = 0, npairs_hi = 0;
    uint32_t qn = 0;            // queued windows (wave-uniform)
    uint32_t since_flush = 0;   // windows since counters were flushed (wave-uniform)
    // counter slot of the held counts (wave-uniform); lanes with cup set hold
    // counts of slot cslot + 1 (the second band of a band-split row block)
    uint32_t cslot = 0;
    bool cup = false;

    auto drain = [&](uint32_t n, const ReqDesc &R) {
        __builtin_amdgcn_wave_barrier();
        if (lane < n) deep_window<SPLIT>(P, queue[qn - n + lane], R, cslot, dcnt, cnt_rep);
        __builtin_amdgcn_wave_barrier();
        qn = uni(qn - n);
    };

    auto flush = [&](const ReqDesc &R) {
        while (qn) drain(qn < (uint32_t)kWave ? qn : (uint32_t)kWave, R);
        const uint64_t cbase = (uint64_t)cslot * P.nc;
        const bool two = SPLIT && __ballot(cup) != 0;
        uint32_t before = npairs + npairs_hi;
#pragma unroll
        for (int k = 0; k < KD; ++k) {
            const uint32_t now = left[k] + left_hi[k];
            const uint32_t v = before - now;
            const uint32_t s = wave_sum(cup ? 0u : v);
            if (lane == 0 && s) atomicAdd(&cnt_rep[cbase + k], (unsigned long long)s);
            if (two) {
                const uint32_t s1 = wave_sum(cup ? v : 0u);
                if (lane == 0 && s1) atomicAdd(&cnt_rep[cbase + P.nc + k], (unsigned long long)s1);
            }
            before = now;
            left[k] = 0;
            left_hi[k] = 0;
        }
        const uint32_t np = npairs + npairs_hi;
        const uint32_t s = wave_sum(cup ? 0u : np);
        if (lane == 0 && s) atomicAdd(&pairs_rep[cslot], (unsigned long long)s);
        if (two) {
            const uint32_t s1 = wave_sum(cup ? np : 0u);
            if (lane == 0 && s1) atomicAdd(&pairs_rep[cslot + 1], (unsigned long long)s1);
        }
        npairs = 0;
        npairs_hi = 0;
        __builtin_amdgcn_wave_barrier();
        const uint32_t ndc = P.n_deep < kDeepCounters ? P.n_deep : kDeepCounters;
        for (uint32_t i = lane; i < ndc; i += kWave) {
            const uint32_t v = dcnt[i];
            if (v) {
                atomicAdd(&cnt_rep[cbase + KD + i], (unsigned long long)v);
                dcnt[i] = 0;
            }
        }
        __builtin_amdgcn_wave_barrier();
        since_flush = 0;
    };

    // The wave's counters hold counts of request req[ri] only: they are
    // flushed when the wave moves on to another request, before a segment
    // that would take them past kFlushWindows windows (before every segment
    // of a band-split request), and once at the end.
    // The descriptor is re-read where needed rather than kept live across
    // the loops.
    uint32_t held = 0;   // counters may hold counts of req[ri] (wave-uniform)
    auto load = [&](uint32_t i) {
        ReqDesc D = P.req[i];
        D.p0 = uni(D.p0); D.p1 = uni(D.p1); D.q0 = uni(D.q0); D.q1 = uni(D.q1);
        D.nrb = uni(D.nrb); D.nwin = uni(D.nwin); D.unit0 = uni64(D.unit0);
        D.rows_p0 = uni(D.rows_p0); D.ip0 = uni(D.ip0);
        D.ulo = uni64(D.ulo); D.ucount = uni64(D.ucount); D.slot = uni(D.slot);
        D.flags = uni(D.flags);
        D.band_rows = uni(D.band_rows); D.band_p0 = uni(D.band_p0);
        return D;
    };

    // How the waves share the units.
    // Workgroup pieces (schedule 0 or 3): pieces of wg_ps units are dealt
    // round-robin to the workgroups, so each workgroup samples the whole launch
    // (rows come grouped by cost); the waves of a workgroup take its units in
    // order through an LDS cursor, in claims of up to a piece that shrink to
    // kMinClaim towards the end of the workgroup's share.  Waves sharing a SIMD
    // progress at unequal rates, so a fixed share per wave leaves the fast ones
    // idle while the slow ones finish; the cursor keeps them all busy to the end
    // and costs one LDS atomic per claim.
    // Round-robin pieces (1): wave w takes pieces w, w + nwaves, ... of up to
    // kPiece units, touching no shared state.
    // Shared counter (2): guided self-scheduling on one global counter, each
    // claim half the remaining units' even share per wave, at least kMinClaim.
    // Its atomics serialise across the device.
    const bool wgshare = P.schedule == 0 || P.schedule == 3;
    const bool guided = P.schedule == 2;
    // about eight pieces per wave, at most kPiece units each (a small launch
    // deals small pieces, so that every wave gets some)
    const uint64_t per_wave = n_units / nwaves / 8;
    const uint64_t psize =
        P.piece ? P.piece : (per_wave < 1 ? 1 : (per_wave < kPiece ? per_wave : kPiece));
    uint64_t piece = w;
    uint64_t lcur = 0, lend = 0;   // the wave's claimed units of its workgroup's share
    // workgroup pieces: at least kWgPieces per workgroup, of up to kPiece units,
    // or of kBigPiece units in launches that fill them (segments of long rows
    // then pay their setup and counter flush less often)
    const uint64_t G = gridDim.x;
    uint64_t wg_ps = n_units / (G * kWgPieces);
    wg_ps = wg_ps >= kBigPiece ? kBigPiece : (wg_ps < 1 ? 1 : (wg_ps < kPiece ? wg_ps : kPiece));
    if (P.piece) wg_ps = P.piece;   // the tuning's own piece size
    for (;;) {
        uint64_t u = 0, uend = 0;
        bool done = false;
        if (wgshare) {
            if (lcur >= lend) {
                const uint64_t n_pieces = (n_units + wg_ps - 1) / wg_ps;
                const uint64_t share =
                    n_pieces > blockIdx.x ? (n_pieces - blockIdx.x + G - 1) / G * wg_ps : 0;
                const uint64_t min_take = wg_ps < kMinClaim ? wg_ps : kMinClaim;
                uint64_t start = 0, take = 0;
                if (lane == 0) {
                    const uint64_t seen = __hip_atomic_load(wg_cursor, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_WORKGROUP);
                    take = (seen < share ? share - seen : 0) / (2 * kWavesPerWG);
                    take = take < min_take ? min_take : (take < wg_ps ? take : wg_ps);
                    start = atomicAdd(wg_cursor, (unsigned long long)take);
                }
                lcur = uni64(start);
                lend = lcur + uni64(take);
                if (lend > share) lend = share;
            }
            if (lcur < lend) {
                // local unit lcur is unit off of the workgroup's j-th piece; a
                // claim may run into the next piece, taken on the next pass
                const uint64_t j = lcur / wg_ps, off = lcur - j * wg_ps;
                const uint64_t n = lend - lcur < wg_ps - off ? lend - lcur : wg_ps - off;
                u = (j * G + blockIdx.x) * wg_ps + off;
                lcur += n;
                // only the launch's last piece can be partial, and it is the
                // last piece of its workgroup
                if (u >= n_units) done = true;
                else uend = n_units - u < n ? n_units : u + n;
            } else {
                done = true;
            }
        } else if (guided) {
            uint64_t start = 0, take = 0;
            if (lane == 0) {
                const uint64_t seen = __hip_atomic_load(P.claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                take = (seen < n_units ? n_units - seen : 0) / (2 * nwaves);
                if (take < kMinClaim) take = kMinClaim;
                start = atomicAdd(P.claim, (unsigned long long)take);
            }
            u = uni64(start);
            take = uni64(take);
            done = u >= n_units;
            if (!done) uend = n_units - u < take ? n_units : u + take;
        } else {
            u = piece * psize;
            done = u >= n_units;
            if (!done) uend = n_units - u < psize ? n_units : u + psize;
            piece += nwaves;
        }
        // request holding unit u: the last i with req[i].unit0 <= u, at or after
        // ri since a wave's pieces only move forward (gallop, then bisect)
        uint32_t lo = ri;
        if (!done) {
            uint32_t step = 1;
            while (lo + step < P.n_req && uni64(P.req[lo + step].unit0) <= u) {
                lo += step;
                step <<= 1;
            }
            uint32_t hi = lo + step < P.n_req ? lo + step : P.n_req;
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (uni64(P.req[mid].unit0) <= u) lo = mid; else hi = mid;
            }
            lo = uni(lo);
        }
        // the counters go out when the wave leaves the request, and at the end
        if (held && (done || lo != ri)) {
            flush(load(ri));
            held = 0;
        }
        if (done) break;
        ri = lo;
        while (u < uend) {
            const ReqDesc R = load(ri);
            const uint64_t rend = R.unit0 + R.ucount;
            const bool past = u >= rend;
            // in a band-split request the next segment's lanes hold other rows
            if (held && (past || since_flush >= kFlushWindows || (SPLIT && (R.flags & kReqBandSplit))))
                flush(R);
            held = 1;
            if (past) {
                held = 0;
                ri = uni(ri + 1);
                continue;
            }
            const uint64_t local = u - R.unit0 + R.ulo;
            const uint32_t rb = uni((uint32_t)(local / R.nwin));
            const uint32_t win0 = uni((uint32_t)(local % R.nwin));
            uint64_t seg_end = R.unit0 + ((uint64_t)(rb + 1) * R.nwin - R.ulo);
            if (seg_end > rend) seg_end = rend;
            if (seg_end > uend) seg_end = uend;
            uint32_t nw = uni((uint32_t)(seg_end - u));
            if (nw > kFlushWindows - since_flush) nw = uni(kFlushWindows - since_flush);

            // ---- segment setup: 64 rows (one per lane), starting column qs ----
            const uint64_t nrows = (uint64_t)R.p1 - R.p0 + 1;
            const uint64_t ridx = (uint64_t)rb * kWave + lane;
            const bool valid = ridx < nrows;
            uint32_t p = 0;
            RowInfo rinfo;
            rinfo.meta = kIdleSubset;
            for (int f = 0; f < kMaxBigFactors; ++f) rinfo.f[f] = 0;
            if (valid) {
                p = R.order ? R.order[ridx] : R.p0 + (uint32_t)ridx;
                // a row order holds only rows of this request; anything else
                // leaves the lane idle rather than indexing outside the row table
                if (p < R.p0 || p > R.p1) {
                    p = 0;
                } else {
                    rinfo = R.rows[p - R.rows_p0];
                    rinfo.meta &= ~8u;
                }
            }
            // counter slot: the request's, or in a band-split request the band
            // of each lane's row (two bands at most in a block of 64 rows)
            if (SPLIT && (R.flags & kReqBandSplit)) {
                const uint32_t band = p ? (p - R.band_p0) / R.band_rows : 0xffffffffu;
                const uint32_t b0 = uni(wave_min(band));
                cslot = uni(R.slot + b0);
                cup = p && band != b0;
            } else {
                cslot = R.slot;
                cup = false;
            }
            const uint32_t nf = (rinfo.meta >> 4) & 15;
            // the wave's largest factor count, from ballots (cross-lane
            // shuffles go through the LDS pipe and cost a round trip each)
            uint32_t nfmax = 0;
    #pragma unroll
            for (int f = 1; f <= MF; ++f)
                if (__ballot(nf >= (uint32_t)f) != 0) nfmax = (uint32_t)f;
            const uint32_t wheel_lane = wheel_byte + (rinfo.meta & 15) * (kWheel * 8);
            const uint32_t qs = R.q0 + win0 * kWave;
            // columns of this lane's row: [q0, q1], cut to region (1.2) in a
            // region; only windows reaching past the wave's tightest bounds need
            // per-lane masks (idle lanes keep the request's bounds: their wheel
            // row already clears every column)
            uint32_t rlo = R.q0, rhi = R.q1;
            if ((R.flags & kReqRegion) && p) {
                const uint32_t a = region_qmin(p), b = 59u * p;
                rlo = a > rlo ? a : rlo;
                rhi = b < rhi ? b : rhi;
            }
            if (p == 1 && rlo < 2) rlo = 2;   // (1, 1) is coprime but p = q
            // in a rectangle every lane has [q0, q1] but the row p = 1, which
            // starts at 2: the wave's bounds need no reduction there
            uint32_t lo_max, hi_min;
            if (R.flags & kReqRegion) {
                lo_max = uni(wave_max(rlo));
                hi_min = uni(wave_min(rhi));
            } else {
                lo_max = (__ballot(p == 1) != 0 && R.q0 < 2) ? 2u : R.q0;
                hi_min = R.q1;
            }
            // a window starting above edge_hi reaches past hi_min; windows
            // k < k_lo start below lo_max and windows k >= k_hi reach past
            // hi_min: only those take the per-lane masks
            const uint32_t edge_hi = hi_min >= (uint32_t)(kWave - 1) ? hi_min - (kWave - 1) : 0;
            const uint32_t k_lo = uni(lo_max > qs ? (lo_max - qs - 1) / kWave + 1 : 0);
            const uint32_t k_hi = uni(edge_hi >= qs ? (edge_hi - qs) / kWave + 1 : 0);

            // dense prime d: the window starting at column qs (offset o = qs mod
            // r) is entry k0 = o / 64 mod r of the lane's row, the following ones
            // k0 + 1, k0 + 2, ...; lb[d] is the lane's byte address of entry kq[d]
            // and every prime moves on by one entry (8 bytes, kk8) per window;
            // every kDenseExt windows kq moves on by kDenseExt mod r, kept below r
            // (entries kq .. kq + kDenseExt - 1 < r + kDenseExt are in the row)
            uint32_t lb[KD + 1], kq[KD + 1];
    #pragma unroll
            for (int k = 0; k < KD; ++k) {
                const uint32_t r = P.dr[k];
                kq[k] = uni(mulr(modr(qs, r, P.dm[k]), P.dinv[k], r, P.dm[k]));
                lb[k] = P.doff[k] + (modr(p, r, P.dm[k]) * (r + kDenseExt) + kq[k]) * 8;
            }
            uint32_t kk8 = 0;   // 8 x window within its group of kDenseExt (wave-uniform)
            uint32_t o30 = uni(qs % kWheel);

            // factor l of p: fo = distance from the window start to the next
            // multiple of l, fd = 64 mod l (64 for l >= 64), fb = LDS byte
            // offset of its pattern entries
            uint32_t fo[MF], fd[MF], fl[MF], fb[MF];
    #pragma unroll
            for (int f = 0; f < MF; ++f) {
                fl[f] = 0; fd[f] = 0; fo[f] = 0xffffffffu;
                fb[f] = pat_byte + kPatSmall * 8;
                if ((uint32_t)f < nfmax && (uint32_t)f < nf) {
                    const uint32_t l = rinfo.f[f];
                    const uint32_t rem = mod_var(qs, l);
                    fl[f] = l;
                    fo[f] = rem ? l - rem : 0;
                    fd[f] = l > (uint32_t)kWave ? (uint32_t)kWave : (uint32_t)kWave % l;
                    if (l < (uint32_t)kWave) fb[f] = pat_byte + c_pat_off[l] * 8;
                }
            }

            // ---- windows ----
            // Window k: columns qb .. qb + 63 of the lane's row.  The wheel word
            // holds the columns coprime to p's factors 2, 3, 5; each factor >= 7
            // clears its multiples; then the dense primes, whose entries for
            // window kk of the current group are kk8 = 8 kk bytes past lb[d].
            const uint32_t nwu = uni(nw);   // keeps the loop exit scalar
            for (uint32_t k = 0; k < nwu; ++k) {
                const uint32_t qb = qs + k * kWave;
                uint64_t alive = lds64(smem, wheel_lane + o30 * 8);
    #pragma unroll
                for (int f = 0; f < MF; ++f) {
                    if ((uint32_t)f < nfmax) {
                        const uint32_t idx = fo[f] < (uint32_t)kWave ? fo[f] : (uint32_t)kWave;
                        alive &= ~lds64(smem, fb[f] + idx * 8);
                        // next window: the distance drops by 64 mod l, or
                        // wraps past a multiple (fo + l - fd < l, no overflow
                        // for any l < 2^32)
                        const uint32_t t = fo[f] - fd[f];
                        fo[f] = fo[f] < fd[f] ? t + fl[f] : t;
                    }
                }
                if (k < k_lo || k >= k_hi) {
                    const uint32_t below = rlo > qb ? rlo - qb : 0;
                    const uint32_t upto = rhi >= qb ? rhi - qb + 1 : 0;
                    alive &= (upto < (uint32_t)kWave ? (1ull << upto) - 1 : ~0ull) &
                             (below < (uint32_t)kWave ? ~0ull << below : 0ull);
                }
                npairs = __builtin_popcount((uint32_t)alive) + npairs;
                npairs_hi = __builtin_popcount((uint32_t)(alive >> 32)) + npairs_hi;
    #pragma unroll
                for (int d = 0; d < KD; ++d) {
                    alive &= ~lds64(smem, lb[d] + kk8);
                    left[d] = __builtin_popcount((uint32_t)alive) + left[d];
                    left_hi[d] = __builtin_popcount((uint32_t)(alive >> 32)) + left_hi[d];
                }
                kk8 += 8;
                if (kk8 == kDenseExt * 8) {
                    // the group is done: fold back to the next group's first
                    // entry, kq + kDenseExt mod r (kept below r)
                    kk8 = 0;
    #pragma unroll
                    for (int d = 0; d < KD; ++d) {
                        kq[d] += P.dext[d];
                        if (kq[d] >= P.dr[d]) {
                            kq[d] -= P.dr[d];
                            lb[d] += (P.dext[d] - P.dr[d]) * 8;
                        } else {
                            lb[d] += P.dext[d] * 8;
                        }
                    }
                }
                o30 += kWave % kWheel;
                if (o30 >= (uint32_t)kWheel) o30 -= kWheel;

                const uint64_t bal = __ballot(alive != 0);
                if (bal) {
                    const uint32_t pos = qn + lane_rank(bal);
                    if (alive) {
                        QEntry e;
                        e.p = p; e.qb = qb; e.mask = alive;
                        queue[pos] = e;
                    }
                    qn = uni(qn + (uint32_t)__popcll(bal));
                    if (qn >= (uint32_t)kWave) drain(kWave, R);
                }
            }
            u += nw;
            since_flush = uni(since_flush + nw);
        }
    }
}

// ---- survivor sort: block bitonic sort of 1024, then rank-based merges ----

__device__ __forceinline__ bool surv_less(const SurvEntry &a, const SurvEntry &b) {
    return a.req < b.req || (a.req == b.req && a.idx < b.idx);
}

constexpr int kSortTile = 1024;

__global__ void __launch_bounds__(256) block_sort_kernel(SurvEntry *a, const unsigned long long *n_dev,
                                                         uint64_t cap) {
    __shared__ SurvEntry s[kSortTile];
    const uint64_t n = *n_dev < cap ? *n_dev : cap;
    const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
    if (base >= n) return;
    for (uint32_t i = threadIdx.x; i < kSortTile; i += blockDim.x) {
        const uint64_t g = base + i;
        if (g < n) {
            s[i] = a[g];
        } else {
            s[i].idx = ~0ull; s[i].req = 0xffffffffu; s[i].pad = 0;
        }
    }
    __syncthreads();
    for (uint32_t k = 2; k <= (uint32_t)kSortTile; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < (uint32_t)kSortTile; i += blockDim.x) {
                const uint32_t ixj = i ^ j;
                if (ixj > i) {
                    const bool up = (i & k) == 0;
                    const SurvEntry x = s[i], y = s[ixj];
                    if (up ? surv_less(y, x) : surv_less(x, y)) { s[i] = y; s[ixj] = x; }
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t i = threadIdx.x; i < kSortTile; i += blockDim.x) {
        const uint64_t g = base + i;
        if (g < n) a[g] = s[i];
    }
}

// The results of a sweep in one launch: out_counts[slot][j] = the sum over
// the n_rep replicas of counter col[j] of the slot (0 where col[j] < 0; the
// canonical counters, j itself, when col is null), out_pairs[slot] = the sum
// of the pair-count replicas, *out_n = the survivor count n; with small_cap
// > 0 and n <= small_cap block 0 also sorts the n survivors into out_surv.
__global__ void __launch_bounds__(256) finish_kernel(
    const unsigned long long *counts, const unsigned long long *pairs, uint32_t n_rep,
    uint64_t stride_c, uint64_t stride_p, const int32_t *col, uint32_t n_slots, uint32_t nc,
    uint32_t np, unsigned long long *out_counts, unsigned long long *out_pairs,
    const unsigned long long *surv_n, unsigned long long *out_n, const SurvEntry *surv,
    uint32_t small_cap, SurvEntry *out_surv) {
    const uint64_t ncount = (uint64_t)n_slots * np, n = ncount + n_slots + 1;
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < n;
         g += (uint64_t)gridDim.x * blockDim.x) {
        if (g < ncount) {
            const uint64_t slot = g / np;
            const uint32_t j = (uint32_t)(g - slot * np);
            const int32_t c = col ? col[j] : (int32_t)j;
            unsigned long long v = 0;
            // (unrolled so that the replica loads are in flight together)
            if (c >= 0) {
    #pragma unroll 8
                for (uint32_t r = 0; r < n_rep; ++r) v += counts[r * stride_c + slot * nc + (uint32_t)c];
            }
            out_counts[g] = v;
        } else if (g < ncount + n_slots) {
            const uint64_t slot = g - ncount;
            unsigned long long v = 0;
    #pragma unroll 8
            for (uint32_t r = 0; r < n_rep; ++r) v += pairs[r * stride_p + slot];
            out_pairs[slot] = v;
        } else {
            *out_n = *surv_n;
        }
    }
    if (blockIdx.x != 0 || small_cap == 0) return;
    __shared__ SurvEntry sv[kSortTile];
    // (more than small_cap survivors are sorted by the caller's own passes)
    const uint64_t m = *surv_n;
    if (m == 0 || m > small_cap) return;
    // bitonic sort over the least power of two >= m (at most kSortTile)
    uint32_t n2 = 2;
    while (n2 < m) n2 <<= 1;
    for (uint32_t i = threadIdx.x; i < n2; i += blockDim.x) {
        if (i < m) {
            sv[i] = surv[i];
        } else {
            sv[i].idx = ~0ull; sv[i].req = 0xffffffffu; sv[i].pad = 0;
        }
    }
    __syncthreads();
    for (uint32_t k = 2; k <= n2; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < n2; i += blockDim.x) {
                const uint32_t ixj = i ^ j;
                if (ixj > i) {
                    const bool up = (i & k) == 0;
                    const SurvEntry x = sv[i], y = sv[ixj];
                    if (up ? surv_less(y, x) : surv_less(x, y)) { sv[i] = y; sv[ixj] = x; }
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) out_surv[i] = sv[i];
}

// Merge sorted runs of length L pairwise.  Keys are distinct, so an element's
// place is its rank in its own run plus the number of smaller keys in the
// partner run.  A pass with L >= n only copies.
__global__ void merge_pass_kernel(const SurvEntry *src, SurvEntry *dst,
                                  const unsigned long long *n_dev, uint64_t cap, uint64_t L) {
    const uint64_t n = *n_dev < cap ? *n_dev : cap;
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < n;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const SurvEntry x = src[g];
        if (L >= n) { dst[g] = x; continue; }
        const uint64_t base = (g / (2 * L)) * (2 * L);
        const uint64_t mid = base + L < n ? base + L : n;
        const uint64_t end = base + 2 * L < n ? base + 2 * L : n;
        uint64_t lo, hi;
        if (g < mid) { lo = mid; hi = end; } else { lo = base; hi = mid; }
        const uint64_t start = lo;
        while (lo < hi) {   // first position whose key is not below x
            const uint64_t m = (lo + hi) >> 1;
            if (surv_less(src[m], x)) lo = m + 1; else hi = m;
        }
        const uint64_t below = lo - start;
        dst[g < mid ? g + below : base + (g - mid) + below] = x;
    }
}

}  // namespace

// a row below 7*11*13*17*19 has at most 4 distinct primes >= 7, below
// 7*11*13*17*19*23 at most 5, any uint32 at most 7
int sweep_factor_slots(uint32_t max_p) {
    return max_p < 323323u ? 4 : (max_p < 7436429u ? 5 : 7);
}

hipError_t launch_sweep(const SweepParams &P, int grid, size_t lds_bytes, uint32_t max_p,
                        hipStream_t s) {
    if (P.K > (uint32_t)kKMax) return hipErrorInvalidValue;
    if (P.n_units == 0 && !P.units_dev) return hipSuccess;
    if (!P.claim) return hipErrorInvalidValue;
    const dim3 g(grid), b(kWave * kWavesPerWG);
    const int mf = sweep_factor_slots(max_p);
#define CUBOID_SWEEP_KS(k, sp)                                                                 \
    if (mf == 4) hipLaunchKernelGGL((sweep_kernel<k, 4, sp>), g, b, lds_bytes, s, P);           \
    else if (mf == 5) hipLaunchKernelGGL((sweep_kernel<k, 5, sp>), g, b, lds_bytes, s, P);      \
    else hipLaunchKernelGGL((sweep_kernel<k, 7, sp>), g, b, lds_bytes, s, P);
#define CUBOID_SWEEP_K(k)                                                                      \
    case k:                                                                                    \
        if (P.band_split) { CUBOID_SWEEP_KS(k, true) } else { CUBOID_SWEEP_KS(k, false) }       \
        break;
    switch (P.K) {
        CUBOID_SWEEP_K(0) CUBOID_SWEEP_K(1) CUBOID_SWEEP_K(2) CUBOID_SWEEP_K(3)
        CUBOID_SWEEP_K(4) CUBOID_SWEEP_K(5) CUBOID_SWEEP_K(6) CUBOID_SWEEP_K(7)
        CUBOID_SWEEP_K(8) CUBOID_SWEEP_K(9) CUBOID_SWEEP_K(10) CUBOID_SWEEP_K(11)
        CUBOID_SWEEP_K(12)
        default: return hipErrorInvalidValue;
    }
#undef CUBOID_SWEEP_K
#undef CUBOID_SWEEP_KS
    return hipGetLastError();
}

hipError_t sweep_max_lds(size_t *bytes) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    int v = 0;
    e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    *bytes = (size_t)v;
    return hipSuccess;
}

hipError_t launch_finish(const unsigned long long *counts, const unsigned long long *pairs,
                         uint32_t n_rep, uint64_t stride_c, uint64_t stride_p, const int32_t *col,
                         uint32_t n_slots, uint32_t nc, uint32_t np, unsigned long long *out_counts,
                         unsigned long long *out_pairs, const unsigned long long *surv_n,
                         unsigned long long *out_n, const SurvEntry *surv, uint64_t small_cap,
                         SurvEntry *out_surv, hipStream_t s) {
    static_assert(kSmallSort == kSortTile, "one sort tile");
    if (small_cap > kSmallSort || (small_cap && (!surv || !out_surv))) return hipErrorInvalidValue;
    const uint64_t n = (uint64_t)n_slots * np + n_slots + 1;
    uint64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(finish_kernel, dim3((unsigned)g), dim3(256), 0, s, counts, pairs, n_rep,
                       stride_c, stride_p, col, n_slots, nc, np, out_counts, out_pairs, surv_n,
                       out_n, surv, (uint32_t)small_cap, out_surv);
    return hipGetLastError();
}

hipError_t launch_sort_surv(SurvEntry *a, SurvEntry *tmp, const unsigned long long *n_dev,
                            uint64_t cap, SurvEntry **out, hipStream_t s) {
    *out = a;
    if (cap == 0) return hipSuccess;
    const uint64_t tiles = (cap + kSortTile - 1) / kSortTile;
    hipLaunchKernelGGL(block_sort_kernel, dim3((unsigned)tiles), dim3(256), 0, s, a, n_dev, cap);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    SurvEntry *src = a, *dst = tmp;
    for (uint64_t L = kSortTile; L < cap; L *= 2) {
        uint64_t g = (cap + 255) / 256;
        if (g > (1u << 16)) g = 1u << 16;
        hipLaunchKernelGGL(merge_pass_kernel, dim3((unsigned)g), dim3(256), 0, s, src, dst, n_dev,
                           cap, L);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        SurvEntry *t = src; src = dst; dst = t;
    }
    *out = src;
    return hipSuccess;
}

}  // namespace cuboid
