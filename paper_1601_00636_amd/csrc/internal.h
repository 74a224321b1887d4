// Internal declarations shared by the host runtime and the HIP kernels of
// libcuboid.  Not part of the public interface (see include/cuboid.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cuboid {

constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kWavesPerWG = 16;      // sweep workgroup = 1024 lanes, one per CU
constexpr int kDenseExt = 16;        // entries past r in each row of a dense window table
constexpr int kKMax = 12;            // most dense (bit-window) primes per launch
constexpr int kMaxBigFactors = 7;    // distinct primes >= 7 of a uint32 (7*11*..*29 < 2^32 < that*31)
constexpr int kQueueCap = 128;       // per-wave queue of windows that outlive the dense primes
constexpr int kDeepCounters = 128;   // per-wave LDS counters for the first deep primes
constexpr int kWheel = 30;           // 2*3*5
constexpr int kWheelSubsets = 9;     // subsets of {2,3,5}, then an all-zero row for idle lanes
constexpr int kIdleSubset = 8;
constexpr int kBucketChunk = 8192;   // rows regrouped by factor count within each chunk
// Multiple patterns: for each prime l in 7..61, l entries (entry d, the
// distance from a window's first column to the next multiple of l, has bit j
// set for every j = d mod l, j < 64); then 65 entries 1<<j (j < 64) and 0,
// used by primes >= 64 whose next multiple is at distance min(d, 64).
constexpr int kPatSmall = 491;       // 7 + 11 + 13 + ... + 61
constexpr int kPatEntries = kPatSmall + 65;

// Distinct prime factors of one row coordinate p.
//   meta bits 0..2: which of 2, 3, 5 divide p; bits 4..7: number of f[] used.
//   f[]: the distinct prime factors >= 7 of p, ascending.
struct RowInfo {
    uint32_t meta;
    uint32_t f[kMaxBigFactors];
};

// One prime tested after the dense phase ("deep" prime).  Its table is kept in
// ratio form: u_r(a, b) = v[a * b^-1 mod r] for a, b != 0, and 0 otherwise.
struct DeepPrime {
    uint32_t r;       // the prime
    uint32_t m;       // floor(2^32 / r), for x mod r by multiply-high
    uint32_t voff;    // byte offset of its ratio vector in the vector pool
    uint32_t ioff;    // element offset of its inverse table in the inverse pool
};

// One rectangle of a launch, with its place in the flattened unit space.
// A unit is one wavefront step: 64 consecutive rows x 64 consecutive columns.
struct ReqDesc {
    uint32_t p0, p1, q0, q1;
    uint32_t nrb;          // ceil(rows / 64)
    uint32_t nwin;         // ceil(cols / 64)
    uint64_t unit0;        // first unit of this request in the flattened order
    uint64_t ulo;          // this launch covers the request's units ulo .. ulo + ucount - 1
    uint64_t ucount;       //   (unit rb * nwin + win: row block rb, column window win)
    uint32_t slot;         // counter slot and survivor tag of the request
    uint32_t flags;        // kReqRegion: per-row columns of region (1.2)
    const RowInfo *rows;   // row info for p at rows[p - rows_p0]
    uint32_t rows_p0;
    uint32_t ip0;          // p0 of the caller's rectangle (survivor indices)
    const uint32_t *order; // rows in processing order, or null for p0, p0 + 1, ...
    const uint8_t *nfac;   // number of f[] of p at nfac[p - rows_p0]
    uint32_t band_rows;    // kReqBandSplit: row p counts into slot
    uint32_t band_p0;      //   slot + (p - band_p0) / band_rows
};

// The columns of row p are min(cbrt(p / 9), p / 59) <= q <= 59 p (Theorem 1.2)
// intersected with [q0, q1], and survivors are tagged p * 2^32 + q.  Needs
// p <= 72796055 so that 59 p < 2^32.
constexpr uint32_t kReqRegion = 1;
// A region request over several report bands of band_rows >= 64 rows, rows in
// natural order: a 64-row block then spans at most two bands, and each lane's
// counts go to the slot of its own row's band.
constexpr uint32_t kReqBandSplit = 2;
constexpr uint32_t kRegionMaxP = 72796055u;

struct SurvEntry {
    uint64_t idx;          // (p - ip0) * (q1 - q0 + 1) + (q - q0); p * 2^32 + q in a region
    uint32_t req;          // slot of the request
    uint32_t pad;
};

struct SweepParams {
    uint32_t K;                          // dense primes in this launch
    uint32_t dr[kKMax];                  // dense prime r
    uint32_t dm[kKMax];                  // floor(2^32 / r)
    uint32_t dinv[kKMax];                // inverse of 64 modulo r
    uint32_t dext[kKMax];                // kDenseExt mod r
    uint32_t doff[kKMax];                // LDS byte offset of that prime's window table
    uint32_t dense_words;                // 64-bit words of all window tables
    const uint64_t *dense_tab;           // window tables in HBM (copied to LDS)
    const uint64_t *wheel;               // 9 x 30 coprimality windows (copied to LDS)
    const uint64_t *patterns;            // multiple patterns (copied to LDS)
    uint32_t n_deep;
    uint32_t nc;                         // counters per request = K + n_deep
    const DeepPrime *deep;
    const uint8_t *vpool;                // ratio vectors
    const uint16_t *ipool;               // inverse tables
    const ReqDesc *req;
    uint32_t n_req;
    uint32_t schedule;                   // 0 or 3 workgroup pieces, 1 round-robin pieces, 2 shared counter
    uint32_t piece;                      // units per piece of schedules 0, 1, 3 (0: chosen by size)
    uint64_t n_units;
    unsigned long long *counts;          // [n_rep][slot][nc], canonical ascending order
    unsigned long long *pairs;           // [n_rep][slot]
    uint32_t n_rep;                      // counter replicas (power of two), by wave
    uint32_t band_split;                 // some request is kReqBandSplit
    uint64_t rep_stride_counts;          // elements between replicas
    uint64_t rep_stride_pairs;
    SurvEntry *surv;
    unsigned long long surv_cap;
    unsigned long long *surv_n;
    const unsigned long long *units_dev; // if set, the unit count is read here, not n_units
    unsigned long long *claim;           // units handed out so far (zero before each launch)
};

// LDS bytes the sweep needs beyond the dense tables.
constexpr size_t kWheelBytes = (size_t)kWheelSubsets * kWheel * 8;
constexpr size_t kQueueEntryBytes = 16;
constexpr size_t kPerWaveBytes = kQueueCap * kQueueEntryBytes + kDeepCounters * 4;
constexpr size_t kPatBytes = (size_t)kPatEntries * 8;
constexpr size_t kWgCtlBytes = 16;   // the workgroup's claim cursor
constexpr size_t kSweepFixedLds =
    kWheelBytes + kPatBytes + kWavesPerWG * kPerWaveBytes + kWgCtlBytes;

// ---- kernel launchers (kernels_*.hip) ----
hipError_t launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t s);
hipError_t launch_copy_u64(uint64_t *dst, const uint64_t *src, uint64_t n, hipStream_t s);
// measured v_bcnt_u32_b32 lane-operations and conflict-free LDS bytes per second
hipError_t run_peak_probes(int cu_count, hipStream_t s, double *valu_lane_ops_per_s,
                           double *lds_bytes_per_s);
hipError_t launch_fill_u8(uint8_t *p, uint64_t n, uint8_t v, hipStream_t s);
hipError_t launch_q_eval(const uint32_t *p, const uint32_t *q, const uint32_t *t,
                         const uint32_t *r, uint64_t n, uint32_t *out, hipStream_t s);
// ratio vectors v_r for primes pr[0..n): v written at vpool + voff[i]
hipError_t launch_ratio_vectors(const uint32_t *pr, const uint32_t *voff, uint32_t n,
                                const uint64_t *work_prefix, uint64_t total_work,
                                uint8_t *vpool, hipStream_t s);
hipError_t launch_inverse_tables(const uint32_t *pr, const uint32_t *ioff, uint32_t n,
                                 const uint64_t *prefix, uint64_t total, uint16_t *ipool,
                                 hipStream_t s);
hipError_t launch_vector_popcount(const uint32_t *pr, const uint32_t *voff, uint32_t n,
                                  const uint8_t *vpool, uint32_t *out, hipStream_t s);
hipError_t launch_pack_table(uint32_t r, const uint8_t *v, const uint16_t *inv, uint8_t *out,
                             hipStream_t s);
hipError_t launch_dense_windows(const uint32_t *pr, const uint32_t *voff, const uint32_t *ioff,
                                const uint32_t *woff, uint32_t n, const uint64_t *prefix,
                                uint64_t total, const uint8_t *vpool, const uint16_t *ipool,
                                uint64_t *out, hipStream_t s);
hipError_t launch_wheel(uint64_t *out, hipStream_t s);
hipError_t launch_patterns(uint64_t *out, hipStream_t s);
uint32_t pattern_offset(uint32_t l);   // entry offset of prime l's patterns (l in 7..61)
hipError_t launch_row_info(const uint32_t *primes16, const uint32_t *magic16, uint32_t n16,
                           uint32_t pstart, uint64_t count, RowInfo *out, uint8_t *nfac,
                           hipStream_t s);
// regroup each request's rows, chunk by chunk, by number of factors >= 7
hipError_t launch_bucket_rows(const ReqDesc *req, uint32_t n_req, const uint64_t *chunk_prefix,
                              uint64_t n_chunks, const uint64_t *row_prefix, uint32_t *order,
                              hipStream_t s, const uint64_t *n_chunks_dev = nullptr,
                              uint32_t grid = 0);
// zero all replicas of the listed counter slots; sum them into out[i][nc + 1]
hipError_t launch_zero_slots(unsigned long long *counts, unsigned long long *pairs,
                             const uint32_t *slots, uint32_t n, uint32_t nc, uint32_t n_rep,
                             uint64_t stride_c, uint64_t stride_p, hipStream_t s);
hipError_t launch_reduce_slots(const unsigned long long *counts, const unsigned long long *pairs,
                               const uint32_t *slots, uint32_t n, uint32_t nc, uint32_t n_rep,
                               uint64_t stride_c, uint64_t stride_p, unsigned long long *out,
                               hipStream_t s);
// dst[i] = sum of n_rep replicas src[r * stride + i], in place on replica 0
hipError_t launch_gather_counts(const unsigned long long *counts, const int32_t *col,
                                uint32_t n_slots, uint32_t nc, uint32_t np,
                                unsigned long long *out, hipStream_t s);
hipError_t launch_reduce_replicas(unsigned long long *buf, uint64_t n, uint32_t n_rep,
                                  uint64_t stride, hipStream_t s);
// zero a[na], b[nb], c[nc] in one launch
hipError_t launch_clear3(uint64_t *a, uint64_t na, uint64_t *b, uint64_t nb, uint64_t *c,
                         uint64_t nc, hipStream_t s);

// max_p: the largest row coordinate of the launch (selects the factor slots)
// factor slots the sweep reserves per row for rows up to max_p (4, 5 or 7)
int sweep_factor_slots(uint32_t max_p);
hipError_t launch_sweep(const SweepParams &P, int grid, size_t lds_bytes, uint32_t max_p,
                        hipStream_t s);
hipError_t sweep_max_lds(size_t *bytes);
// sorts n <= cap entries (n read from device) ascending by (req, idx) into out
hipError_t launch_sort_surv(SurvEntry *a, SurvEntry *tmp, const unsigned long long *n_dev,
                            uint64_t cap, SurvEntry **out, hipStream_t s);
// Replica sums, counts in the caller's order (col, or canonical when null) and
// the survivor count n, in one launch: out_counts[n_slots][np],
// out_pairs[n_slots], *out_n; with small_cap (<= kSmallSort) and
// n <= small_cap also the n survivors of surv, sorted, into out_surv.
constexpr uint64_t kSmallSort = 1024;
hipError_t launch_finish(const unsigned long long *counts, const unsigned long long *pairs,
                         uint32_t n_rep, uint64_t stride_c, uint64_t stride_p, const int32_t *col,
                         uint32_t n_slots, uint32_t nc, uint32_t np, unsigned long long *out_counts,
                         unsigned long long *out_pairs, const unsigned long long *surv_n,
                         unsigned long long *out_n, const SurvEntry *surv, uint64_t small_cap,
                         SurvEntry *out_surv, hipStream_t s);

// ---- root check (kernels_roots.hip) ----
struct RootCand {
    uint32_t p, q;
    uint32_t nf;           // distinct primes of the constant's square root
    uint32_t pad;
    uint32_t fp[20];       // those primes
    uint32_t fe[20];       // exponents (in p^5 q^5, or p^4 / q^4 on an axis)
    uint64_t bound_lo;     // every positive root t is <= bound (128 bits:
    uint64_t bound_hi;     // about 2^66.5 at p, q near 2^32)
    uint64_t ndiv;         // number of divisors (saturating)
};
struct RootHit {
    uint32_t cand;         // index of the pair
    uint32_t pad;
    uint64_t t_lo, t_hi;   // the candidate t = t_hi 2^64 + t_lo
};
hipError_t launch_root_factor(const uint32_t *p, const uint32_t *q, uint64_t n,
                              const uint32_t *primes16, const uint32_t *magic16, uint32_t n16,
                              RootCand *out, hipStream_t s);
hipError_t launch_root_eval(const RootCand *c, uint64_t n_cand, const uint64_t *prefix,
                            uint64_t w0, uint64_t nwork, RootHit *hits, uint64_t cap,
                            unsigned long long *n_hits, hipStream_t s);

}  // namespace cuboid
