/*
 * cuboid.h — C interface of the MI355X (gfx950) modulo-primes sieve for
 * perfect cuboids (second cuboid conjecture).
 *
 * The method is that of R.R. Gallyamov, I.R. Kadyrov, D.D. Kashelevskiy,
 * N.G. Kutlugallyamov, R.A. Sharipov, "A fast modulo primes algorithm for
 * searching perfect cuboids and its implementation", arXiv:1601.00636:
 *
 *   - Q_pq(t) is the even tenth-degree polynomial of eq. (1.1);
 *   - a pair (p~, q~) of residues modulo a prime r is "unsolvable" when no
 *     t~ in [0, r) makes Q_{p~q~}(t~) vanish modulo r (Definition 1.1); the
 *     unsolvability bit u_r(p~, q~) of eq. (2.3) is 1 for such pairs;
 *   - a pair (p, q) for which some sieve prime r has u_r(p mod r, q mod r) = 1
 *     has no integer root t (section 2) and is rejected; the rest survive;
 *   - by Theorem 1.1 a perfect cuboid of this family needs a positive integer
 *     root t of Q_pq with t > p^2, t > pq, t > q^2, (p^2 + t)(pq + t) > 2t^2.
 *
 * Conventions for every function below:
 *   - Return value: a cuboid_status code (0 = CUBOID_OK) unless stated.  The
 *     numbering reuses the paper's return codes where the meaning matches
 *     (section 5: 1 = already running / busy, 6 = tables not loaded).
 *   - Buffers: all pointers are HOST memory owned by the caller, unless a
 *     parameter says "device".  The library never keeps a caller pointer after
 *     the call returns (the server holds each ticket's results itself until
 *     they are polled).
 *   - The library owns the context, its device tables and device scratch.
 *   - `hip_stream` is a hipStream_t (as void*); NULL means the context's own
 *     stream.  Calls that return host results synchronise that stream before
 *     returning.
 *   - Misuse (null pointers, destroyed context, bad ranges) is reported by a
 *     status code and never crashes, as the paper's DLL promises (section 5).
 *   - One context may be used from several host threads; calls on one context
 *     are serialised internally.
 */
#ifndef CUBOID_H
#define CUBOID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum cuboid_status {
    CUBOID_OK = 0,
    CUBOID_E_BUSY = 1,        /* work in flight, or a server still running       */
    CUBOID_E_RANGE = 2,       /* empty/inverted bounds or a bound equal to 0      */
    CUBOID_E_LIMIT = 3,       /* a size limit exceeded (see each function)        */
    CUBOID_E_PRIMES = 4,      /* prime list: empty, non-prime, duplicate, >= 2^16 */
    CUBOID_E_CAPACITY = 5,    /* output buffer too small; required size returned  */
    CUBOID_E_NOT_LOADED = 6,  /* null or destroyed context                        */
    CUBOID_E_DEVICE = 7,      /* no usable gfx950 device, or a HIP runtime error  */
    CUBOID_E_ARG = 8,         /* null pointer or invalid argument                 */
    CUBOID_E_IO = 9,          /* a file could not be opened, read or written      */
    CUBOID_E_DATA = 10        /* file contents differ from the tables they name   */
} cuboid_status;

/*
 * A context handle is an opaque token, not an address: it names a slot of the
 * library's context table and the generation of that slot, so the handle of
 * a destroyed context is refused (E_NOT_LOADED) for the rest of the process,
 * even after new contexts are created.  Every call holds its context for its
 * whole length; cuboid_destroy returns E_BUSY meanwhile.
 */
typedef struct cuboid_ctx cuboid_ctx;

/* Short English text for a status code (static storage). */
const char *cuboid_status_string(int status);

/* Library version string, e.g. "0.1.0 gfx950" (static storage). */
const char *cuboid_version(void);

/*
 * Create a context on HIP device `hip_device`: allocates the constant device
 * tables (small-prime list, coprimality wheel).  Unsolvability tables are
 * built on the GPU the first time a prime set is used and then stay resident
 * (the analogue of the paper's Load_Cuboid_Binaries, section 4).
 * Errors: E_ARG (out == NULL), E_DEVICE (no device / not gfx950 / HIP error),
 * E_LIMIT (4096 contexts alive at once).
 */
int cuboid_create(cuboid_ctx **out, int hip_device);

/*
 * Destroy a context and free its device memory (cf. Release_Cuboid_Binaries,
 * section 5).  Returns E_BUSY, destroying nothing, while a call (running or
 * waiting for the context), a server or a search is still using it;
 * E_NOT_LOADED for NULL, a destroyed context or any other value.
 */
int cuboid_destroy(cuboid_ctx *ctx);

/*
 * Evaluate Q_pq(t) mod r (eq. 1.1 reduced as in eq. 2.2) on the GPU for n
 * quadruples: out[i] = Q_{p[i] q[i]}(t[i]) mod r[i].  The analogue of the
 * paper's Calculate_Q_pq_mod_prime (section 3), which handles 16-bit moduli.
 * p, q, t: any uint32; r: 2 <= r < 65536 (any integer, prime or not).
 * Errors: E_ARG (null pointer with n > 0, an r out of range), E_DEVICE.
 */
int cuboid_q_mod_prime(cuboid_ctx *ctx, const uint32_t *p, const uint32_t *q,
                       const uint32_t *t, const uint32_t *r, uint64_t n, uint32_t *out);

/*
 * The unsolvability table u_r of eq. (2.3) for one prime r, built on the GPU,
 * in the byte packing of eq. (2.6): bit a*r + b holds u_r(a, b) (a = p~ row,
 * b = q~ column), eight bits per byte least-significant first, the last byte
 * zero-padded; ceil(r*r/8) bytes.
 * *written receives the byte count (also when cap is too small).
 * Errors: E_PRIMES (r not a prime below 65536), E_CAPACITY (cap too small),
 * E_ARG, E_DEVICE.
 */
int cuboid_table_bytes(cuboid_ctx *ctx, uint32_t r, uint8_t *out, size_t cap, size_t *written);

/*
 * The sieve over the rectangle p0 <= p <= p1, q0 <= q <= q1 (inclusive,
 * uint32 coordinates >= 1).
 *
 * Domain: pairs with p != q and gcd(p, q) = 1 (Conjecture 1.1); their number is
 * written to *n_pairs.  A pair is rejected by the FIRST prime r, in ascending
 * order of the prime list, with u_r(p mod r, q mod r) = 1, and counts[i] (for
 * primes[i]) counts the pairs so rejected; primes whose table is all zero
 * (2, 3, 5, 7: section 2) always count 0.  The primes may be given in any
 * order; counts[] follows the order given.
 * Survivors (pairs no prime rejects) are written to survivors[] as ascending
 * uint64 indices (p - p0) * (q1 - q0 + 1) + (q - q0); *n_survivors receives
 * their number.  sum(counts) + *n_survivors == *n_pairs always.
 *
 * primes: 1 <= n_primes <= 6542 distinct primes, each < 65536.
 * survivors may be NULL when cap == 0.
 * Errors: E_RANGE (p0 > p1, q0 > q1, or p0 == 0 or q0 == 0), E_PRIMES,
 * E_CAPACITY (more than cap survivors: *n_survivors is set to the number
 * needed, counts/n_pairs are valid, survivors[] contents are unspecified),
 * E_LIMIT (unsolvability tables for the prime set exceed the device budget),
 * E_ARG, E_DEVICE, E_NOT_LOADED.
 */
int cuboid_sieve_range(cuboid_ctx *ctx, uint32_t p0, uint32_t p1, uint32_t q0, uint32_t q1,
                       const uint32_t *primes, uint32_t n_primes,
                       uint64_t *survivors, uint64_t cap, uint64_t *n_survivors,
                       uint64_t *counts, uint64_t *n_pairs, void *hip_stream);

/*
 * The sieve over region (1.2) of Theorem 1.2 for p0 <= p <= p1, the scan of
 * sections 5 and 6: for each p every integer q with
 * min(cbrt(p / 9), p / 59) <= q <= 59 p (the lower bound taken exactly: the
 * smaller of the least q with 9 q^3 >= p and the least q with 59 q >= p), in
 * the domain and with the first-rejecter counting of cuboid_sieve_range.
 *
 * Survivors are written as ascending uint64 values p * 2^32 + q.
 * r_max (may be NULL) receives one value per report band of band_rows
 * consecutive p starting at p0 (ceil((p1 - p0 + 1) / band_rows) entries; the
 * paper reports per hundred): the largest prime some pair of the band was
 * tested against, i.e. its deepest first rejecting prime, or the largest
 * listed prime if a pair of the band passed every prime, or 1 if the band
 * holds no pair.  The largest r_max over the bands is the depth the sieve
 * reached (section 6: 137 for p <= 154000 with the primes 11..541).
 *
 * Limits: 1 <= p0 <= p1 <= 72796055 (so that 59 p < 2^32, the paper's 32-bit
 * bound of section 6), band_rows >= 1.
 * Errors: E_RANGE (p0 == 0 or p0 > p1), E_LIMIT (p1 > 72796055, or more
 * survivors than the device list holds), E_ARG (band_rows == 0, a required
 * pointer NULL), E_PRIMES, E_CAPACITY (as in cuboid_sieve_range), E_DEVICE,
 * E_NOT_LOADED.
 */
int cuboid_sieve_region(cuboid_ctx *ctx, uint32_t p0, uint32_t p1, uint32_t band_rows,
                        const uint32_t *primes, uint32_t n_primes,
                        uint64_t *survivors, uint64_t cap, uint64_t *n_survivors,
                        uint64_t *counts, uint64_t *n_pairs, uint32_t *r_max, void *hip_stream);

/*
 * One positive integer root of Q_pq (eq. 1.1) confirmed in exact arithmetic.
 * flags: bit 0 t > p^2, bit 1 t > pq, bit 2 t > q^2,
 *        bit 3 (p^2 + t)(pq + t) > 2 t^2  (the inequalities of Theorem 1.1);
 * all four set means (p, q, t) yields a perfect cuboid.
 */
typedef struct cuboid_root {
    uint32_t p, q;
    uint64_t t;             /* the root t = t_hi 2^64 + t: low 64 bits       */
    uint64_t t_hi;          /* high bits (candidates reach about 2^66.5 for  */
                            /* p, q near 2^32; every root found so far,       */
                            /* t = p^2 for p = q or q = 0, is below 2^64)     */
    uint32_t flags;
    uint32_t input_index;   /* position of (p, q) in the input arrays */
} cuboid_root;

/*
 * Exact integer-root check for n pairs (typically sieve survivors).
 * For every i, all integers t > 0 with Q_{p[i] q[i]}(t) = 0 are reported.
 * GPU part: t^2 divides the constant term p^10 q^10 of Q as a polynomial in
 * t^2 (p^8 or q^8 when the other is 0), so t runs over the divisors of
 * p^5 q^5 up to a root bound; each candidate is evaluated modulo three 62-bit
 * primes.  CPU part: candidates that vanish modulo all three are confirmed in
 * exact multiprecision arithmetic.  Roots are listed by input index, then by t.
 * Any p[i], q[i] < 2^32 (the sieve's whole coordinate range, up to q = 59 p
 * at the paper's p_max, sections 5-6): the root bound on t is then below
 * 2^67, and candidates are carried in 128 bits.  p[i] = q[i] = 0 has no
 * positive roots.
 * Errors: E_LIMIT (more than 2^40 candidates for one pair), E_CAPACITY
 * (*n_roots set to the number needed), E_ARG, E_DEVICE, E_NOT_LOADED.
 */
int cuboid_root_check(cuboid_ctx *ctx, const uint32_t *p, const uint32_t *q, uint64_t n,
                      cuboid_root *roots, uint64_t cap, uint64_t *n_roots);

/*
 * Exact CPU confirmation alone (no GPU): *is_root = 1 iff Q_pq(t) == 0 in
 * exact integer arithmetic, for t = t_hi 2^64 + t_lo; *flags as in
 * cuboid_root.  Any p, q < 2^32; t < 2^70.
 * Errors: E_ARG, E_LIMIT (t >= 2^70).
 */
int cuboid_exact_check(uint32_t p, uint32_t q, uint64_t t_lo, uint64_t t_hi, int *is_root,
                       uint32_t *flags);

/*
 * Q_pq(t) in exact integer arithmetic on the CPU, t = t_hi 2^64 + t_lo, as a
 * signed decimal string with its terminating NUL (for checking the exact
 * arithmetic).  Any p, q < 2^32; t < 2^70.
 * Errors: E_ARG, E_LIMIT (t >= 2^70), E_CAPACITY (cap too small for the
 * string).
 */
int cuboid_exact_value(uint32_t p, uint32_t q, uint64_t t_lo, uint64_t t_hi, char *out,
                       size_t cap);

/*
 * Prime-list canonicalisation alone (no GPU): validates `primes` and writes
 * them in ascending order to sorted_out[n] and, for each, whether its table is
 * known to be all zero by the paper's statement (2, 3, 5, 7: section 2) to
 * trivial_out[n] (may be NULL).  Errors: E_PRIMES, E_ARG.
 */
int cuboid_canonical_primes(const uint32_t *primes, uint32_t n, uint32_t *sorted_out,
                            uint8_t *trivial_out);

/* ------------------------------------------------------------------ batched */

typedef struct cuboid_request {
    uint32_t p0, p1, q0, q1;      /* inclusive rectangle, coordinates >= 1 */
} cuboid_request;

typedef struct cuboid_result {
    uint64_t *survivors;          /* caller buffer, ascending indices as in cuboid_sieve_range */
    uint64_t cap;                 /* its capacity                                  */
    uint64_t n_survivors;         /* out: number of survivors (may exceed cap)      */
    uint64_t *counts;             /* caller buffer [n_primes], order of the prime list */
    uint64_t n_pairs;             /* out                                            */
    int32_t status;               /* out: CUBOID_OK, CUBOID_E_CAPACITY or CUBOID_E_RANGE */
    uint32_t reserved;
} cuboid_result;

/*
 * Many rectangles in one persistent launch: every request's outputs are those
 * cuboid_sieve_range would give for it alone (bit-exact).  Work is split into
 * 64-row x 64-column units shared out over the whole GPU regardless of
 * request sizes.  Returns E_CAPACITY if any request's status is E_CAPACITY
 * (the others are complete); an invalid rectangle sets that request's status
 * to E_RANGE and fails the call with E_RANGE before any work.  Returns E_LIMIT
 * (with every n_survivors still exact) if the survivors of the whole batch
 * exceed 2^26.
 * Errors: as cuboid_sieve_range, plus E_ARG for n_req == 0 or NULL arrays.
 */
int cuboid_sieve_batch(cuboid_ctx *ctx, const cuboid_request *req, uint32_t n_req,
                       const uint32_t *primes, uint32_t n_primes,
                       cuboid_result *res, void *hip_stream);

/*
 * cuboid_sieve_batch with the results left in device memory, for callers whose
 * next step runs on the GPU (and to time the sieve without the PCIe transfer
 * of its results).  The rectangles are read from host memory (16 bytes each,
 * staged with the launch).  Device buffers, owned by the caller (from
 * cuboid_device_alloc, or hipMalloc of the HIP runtime this library links):
 *   counts_dev     [n_req][n_primes] uint64, the order of the prime list
 *   pairs_dev      [n_req] uint64, coprime pairs p != q of each rectangle
 *   survivors_dev  surv_cap entries of 16 bytes {uint64 idx; uint32 req;
 *                  uint32 0}, sorted by (req, idx); idx as in
 *                  cuboid_sieve_range for rectangle req
 * *n_survivors (host) receives the total.  Beyond surv_cap the list holds the
 * first surv_cap in that order and the call returns E_CAPACITY; counts and
 * pairs are complete either way.  E_LIMIT if more than 2^26 survive (counts
 * and pairs complete, the list unspecified).  Returns after the results are
 * in place.  Errors: E_ARG (NULL arrays, n_req == 0), E_RANGE (an invalid
 * rectangle, before any work), E_PRIMES, E_DEVICE, E_NOT_LOADED.
 */
int cuboid_sieve_batch_dev(cuboid_ctx *ctx, const cuboid_request *req, uint32_t n_req,
                           const uint32_t *primes, uint32_t n_primes, uint64_t *counts_dev,
                           uint64_t *pairs_dev, void *survivors_dev, uint64_t surv_cap,
                           uint64_t *n_survivors, void *hip_stream);

/*
 * cuboid_sieve_batch_dev for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, results and errors, but the call allocates no
 * device or pinned memory.  Its device scratch (descriptors, row order,
 * counter replicas, survivor list and sort buffer, the survivor count) is
 * one fixed array of 64 MiB per GPU inside the library, held until the
 * process ends; every call on a GPU shares it, and the library makes those
 * calls take turns (each holds the array until its work has completed), so
 * they never overlap on it.  Every counter it needs is cleared by each call.
 * Requirements and limits:
 *   - the prime list's tables and the resident row table up to the largest
 *     p1 must exist: any earlier sieve call on this context with the same
 *     prime list and rows at least as far builds them (a one-pair
 *     cuboid_sieve_range at (p1, 1) does); otherwise E_NOT_LOADED;
 *   - p1 <= 2^24 (E_LIMIT beyond), launched call by call (no graph);
 *   - E_LIMIT when the requests' descriptors and one set of counters do not
 *     fit the array with room for 1024 survivors (about 75 000 requests at
 *     94 primes), or when more survivors arise than the array holds (up to
 *     2^19; counts and pairs are complete, the list unspecified).
 * Rows of the largest requests keep their natural order once 6.3 million
 * regrouped rows fill the array's row-order part (results are unchanged).
 */
int cuboid_sieve_batch_dev_noalloc(cuboid_ctx *ctx, const cuboid_request *req, uint32_t n_req,
                                   const uint32_t *primes, uint32_t n_primes,
                                   uint64_t *counts_dev, uint64_t *pairs_dev,
                                   void *survivors_dev, uint64_t surv_cap,
                                   uint64_t *n_survivors, void *hip_stream);

/*
 * Device memory on the context's GPU for the _dev entry points, and a
 * synchronous copy back to host memory (on hip_stream, NULL = the context's
 * stream).  cuboid_device_free waits for the context's stream first; NULL is a
 * no-op.  Errors: E_ARG (bytes == 0 for alloc, NULL pointers), E_DEVICE.
 */
int cuboid_device_alloc(cuboid_ctx *ctx, size_t bytes, void **out);
/*
 * Measured peaks of the context's GPU for the sweep's roofline: lane-
 * operations per second of v_bcnt_u32_b32 over 8 independent chains per lane
 * at full occupancy, and bytes per second of conflict-free 64-bit LDS reads
 * (8 workgroups of 256 lanes per compute unit, a few milliseconds each).
 * Errors: E_ARG (NULL outputs), E_DEVICE.
 */
int cuboid_probe_peaks(cuboid_ctx *ctx, double *valu_lane_ops_per_s, double *lds_bytes_per_s);
int cuboid_device_free(cuboid_ctx *ctx, void *p);
int cuboid_device_read(cuboid_ctx *ctx, void *dst, const void *src_dev, size_t bytes,
                       void *hip_stream);

/* ------------------------------------------------------------------ served */

/*
 * A request server over one context and one prime list: a worker thread
 * keeps the unsolvability tables resident and runs continuous batching.
 * Requests submitted while others are on the GPU are admitted as counter
 * slots and device memory free up and join the next launch; every launch
 * takes at most `max_launch_units` 64 x 64 units from the requests admitted
 * to its stream (a large request spans several launches), so small requests
 * are not held behind large ones.  Each request's results are bit-exact those
 * of cuboid_sieve_range alone.  Survivors of a launch go to a device pool per
 * stream (2^16 entries at first); a launch that overflows it is swept again
 * with the pool grown to hold them all (up to 2^26), so survivor lists are
 * complete.  Rows beyond the resident row table (p above 2^24, up to
 * 2^32 - 1) get their factor lists computed per request into the device
 * arena.
 */
typedef struct cuboid_server cuboid_server;

typedef struct cuboid_server_config {
    uint32_t streams;             /* launches in flight at once (0 = 2)                  */
    uint32_t max_slots;           /* requests admitted at once (0 = 4096)                */
    uint64_t max_launch_units;    /* units per launch (0 = 2^22)                         */
    uint64_t hbm_budget_bytes;    /* device memory for per-request row orders; 0 = a      */
                                  /* quarter of the free device memory, 64 MiB .. 4 GiB   */
} cuboid_server_config;

typedef struct cuboid_server_stats {
    uint64_t submitted, completed, launches, units;
    uint32_t max_admitted;        /* most requests admitted at the same time        */
    uint32_t resweeps;            /* launches swept again after a survivor overflow */
} cuboid_server_stats;

typedef struct cuboid_request_timing {
    uint64_t submit_ns, admit_ns, done_ns;   /* steady clock, nanoseconds */
} cuboid_request_timing;

/*
 * Start a server.  primes as in cuboid_sieve_range.  cfg may be NULL.
 * While a server runs, cuboid_destroy on its context returns E_BUSY.
 * Errors: E_PRIMES, E_ARG, E_DEVICE, E_NOT_LOADED.
 */
int cuboid_server_start(cuboid_ctx *ctx, const uint32_t *primes, uint32_t n_primes,
                        const cuboid_server_config *cfg, cuboid_server **out);

/*
 * Queue one rectangle; *ticket identifies it.  Returns at once.  A request
 * whose own row table (33 bytes per row, for p1 above 2^24) exceeds the
 * whole arena, or one of whose launches leaves more than 2^26 survivors,
 * finishes with status E_LIMIT (counts and pairs still exact in the second
 * case).  Errors: E_RANGE (invalid rectangle), E_BUSY (stopping).
 */
int cuboid_server_submit(cuboid_server *srv, const cuboid_request *req, uint64_t *ticket);

/*
 * Queue n rectangles at once (one lock, one wake-up of the server), as n
 * calls of cuboid_server_submit would: tickets[i] identifies req[i].  All or
 * none are queued: an invalid rectangle queues none and returns E_RANGE with
 * *bad set to its index (bad may be NULL).  Errors: E_ARG (n = 0 or a null
 * pointer), E_RANGE, E_BUSY (stopping).
 */
int cuboid_server_submit_many(cuboid_server *srv, const cuboid_request *req, uint32_t n,
                              uint64_t *tickets, uint32_t *bad);

/*
 * Results of a ticket into res (counts[n_primes], survivors up to res->cap,
 * n_survivors, n_pairs, status).  wait = 0 returns E_BUSY when not finished;
 * wait != 0 blocks until it is.  A ticket's results are handed out once:
 * after a successful poll the ticket is forgotten.  E_CAPACITY leaves the
 * results in place (n_survivors set) so the caller can poll again with room.
 * timing may be NULL.  Errors: E_ARG (unknown ticket), E_BUSY, E_CAPACITY.
 */
int cuboid_server_poll(cuboid_server *srv, uint64_t ticket, cuboid_result *res, int wait,
                       cuboid_request_timing *timing);

int cuboid_server_stats_get(cuboid_server *srv, cuboid_server_stats *out);

/* Finish every admitted and pending request, stop the worker, free the server. */
int cuboid_server_stop(cuboid_server *srv);

/* ------------------------------------------------------------------ tuning */

typedef struct cuboid_tuning {
    uint32_t dense_primes;   /* K: leading non-trivial primes tested as 64-wide bit windows */
    uint32_t workgroups;     /* persistent grid size (0 = one per compute unit) */
    uint32_t lds_budget;     /* bytes of LDS allowed for the dense windows
                                (0 = all that a workgroup has left)         */
    uint32_t schedule;       /* how waves share a launch's units: 0 or 3 =
                                workgroup pieces (pieces dealt round-robin to
                                the workgroups, taken by their waves through an
                                LDS cursor), 1 = round-robin pieces per wave,
                                2 = one shared counter in device memory;
                                results never depend on it                    */
    uint32_t piece_units;    /* 64x64 units per piece of schedules 0, 1 and 3
                                (0 = chosen from the launch size: up to 256,
                                or 4096 in launches of more than 32 x 4096
                                units per workgroup); at most 2^20            */
} cuboid_tuning;

/*
 * Time candidate tunings for `primes` on a sample rectangle of 32768 x 65536
 * pairs near 2^19 and keep the fastest for this context: first the last six
 * dense-prime counts that fit in LDS times grids of 1, 2, 4 and 8 workgroups
 * per compute unit, then for the best of those the work sharing (workgroup
 * pieces of 64, 128, 512, 1024 or 4096 units or chosen by size, round-robin
 * pieces per wave, the shared counter).  If cache_path is non-NULL the choice
 * (every field) is read from / appended to that JSON-lines file, keyed by
 * device architecture and prime set.  Results never depend on the tuning.
 * out may be NULL.
 */
int cuboid_autotune(cuboid_ctx *ctx, const uint32_t *primes, uint32_t n_primes,
                    const char *cache_path, cuboid_tuning *out);

/*
 * As cuboid_autotune, but timed on the caller's own requests: a batch that
 * stands for the workload to come (the same rectangles as cuboid_sieve_batch
 * takes; the sample is swept several times per candidate, so a few tens of
 * milliseconds of work is plenty).  The cache key adds a hash of the sample.
 * Errors: E_ARG (no sample), E_RANGE (a rectangle is invalid), E_PRIMES.
 */
int cuboid_autotune_for(cuboid_ctx *ctx, const uint32_t *primes, uint32_t n_primes,
                        const cuboid_request *sample, uint32_t n_sample,
                        const char *cache_path, cuboid_tuning *out);

/* Set (NULL = restore defaults) or read the tuning used for `primes`. */
int cuboid_set_tuning(cuboid_ctx *ctx, const uint32_t *primes, uint32_t n_primes,
                      const cuboid_tuning *tuning);
int cuboid_get_tuning(cuboid_ctx *ctx, const uint32_t *primes, uint32_t n_primes,
                      cuboid_tuning *out);

/* ------------------------------------------------------------- table files */

/*
 * The paper's binary table files (section 2, eq. 2.7; section 3
 * Write_pq_file_stream; section 4 Load_Cuboid_Binaries).
 *
 * tables file: the packed tables u_r of the primes, ascending, one after the
 *   other, each in the layout of eq. (2.6) (ceil(r*r/8) bytes).
 * primes file: one 8-byte item per prime, as the paper's C++ struct
 *   {short prime; unsigned int p_offset;} lays out on x86: int16 prime
 *   (little-endian), 2 zero bytes of padding, uint32 byte offset of its table
 *   in the tables file (little-endian).
 * text file (may be NULL): each table as "r = <r>" followed by r lines of r
 *   space-separated 0/1 digits (row p~, column q~, as printed in eq. 2.5) and
 *   an empty line.
 * The primes must be below 32768 (int16) and the tables must fit 2^32 bytes,
 * the bound (2.7) (in practice r < 9697).
 * Errors: E_PRIMES, E_LIMIT (a prime >= 32768 or tables beyond 2^32 bytes),
 * E_IO, E_DEVICE, E_NOT_LOADED, E_ARG.
 */
int cuboid_write_table_files(cuboid_ctx *ctx, const uint32_t *primes, uint32_t n_primes,
                             const char *tables_path, const char *primes_path,
                             const char *text_path);

/*
 * Reads a tables file and a primes file in the format above and checks them
 * bit for bit against the tables computed on the device; on success writes
 * the primes (in file order) to primes_out and their number to *n_primes.
 * Errors: E_IO (missing, unreadable or truncated file), E_DATA (offsets not
 * contiguous from 0, padding not zero, or a table that differs), E_PRIMES (an
 * entry that is not a prime, or a repeated prime), E_CAPACITY (cap smaller
 * than the number of primes; *n_primes set), E_DEVICE, E_NOT_LOADED, E_ARG.
 */
int cuboid_check_table_files(cuboid_ctx *ctx, const char *tables_path, const char *primes_path,
                             uint32_t *primes_out, uint32_t cap, uint32_t *n_primes);

/* ------------------------------------------------------------------ search */

/*
 * Resumable background search over region (1.2), after the search loop of
 * section 5 (Start_searching, Get_current_p, Get_current_r_max,
 * Stop_searching).  A host thread scans, from row p and column q on, every
 * row p' <= p_end with the columns of (5.2), min(cbrt(p'/9), p'/59) <= q' <=
 * 59 p', through the same sieve as cuboid_sieve_region.
 */
typedef struct cuboid_search cuboid_search;   /* opaque, owned by the library */

typedef struct cuboid_search_report {
    uint32_t p, q;          /* next pair to scan (row p from column q); after a */
                            /* stop, the exit point to restart from             */
    uint32_t p_hundred;     /* p rounded down to a multiple of 100 (the paper's */
                            /* Get_current_p)                                   */
    uint32_t r_max;         /* largest prime used in the last hundred of p      */
                            /* scanned; 1 again at each new hundred             */
    uint64_t pairs;         /* coprime pairs scanned since the start            */
    uint64_t survivors;     /* pairs no prime rejected since the start          */
    int64_t unix_time;      /* when this report was taken, seconds              */
    int32_t running;        /* 1 while the search thread runs                   */
    int32_t status;         /* CUBOID_OK, or the error that ended the search    */
} cuboid_search_report;

/*
 * Starts the search thread and returns at once (section 5: Start_searching,
 * whose first call is Start_searching(152, 3)).  p_end = 0 means up to
 * 72796055, the last p with 59 p < 2^32.  report_path (may be NULL) names a
 * text file that cuboid_search_stop appends its report line to.  One search
 * per context at a time; the context cannot be destroyed while it runs.
 * Errors: E_BUSY (a search is running on ctx), E_RANGE (p < 152, q outside
 * (5.2) for row p, or p_end < p), E_LIMIT (p > 72796055), E_PRIMES,
 * E_NOT_LOADED, E_ARG.
 */
int cuboid_search_start(cuboid_ctx *ctx, const uint32_t *primes, uint32_t n_primes, uint32_t p,
                        uint32_t q, uint32_t p_end, const char *report_path,
                        cuboid_search **out);
/* Progress (section 5: Get_current_p, Get_current_r_max), any time. */
int cuboid_search_current(cuboid_search *s, cuboid_search_report *out);
/* Pairs that passed every prime so far, as ascending p * 2^32 + q (the first
 * 2^20 kept); *n gets their number; E_CAPACITY if cap is smaller. */
int cuboid_search_survivors(cuboid_search *s, uint64_t *pq, uint64_t cap, uint64_t *n);
/*
 * Stops at the next row boundary (or takes the finished search), writes the
 * final report to *out (may be NULL), appends to the report file the time
 * stamp line and "Stop with p=<p>, q=<q>, r_max=<r_max>" (section 5), frees
 * the search and returns its status.  Restarting from report.p, report.q
 * continues without gap or overlap.
 */
int cuboid_search_stop(cuboid_search *s, cuboid_search_report *out);

/* ------------------------------------------------------------------ timing */

typedef struct cuboid_timing {
    double sweep_ms;         /* sieve sweep kernel, HIP events on the call's stream */
    double total_gpu_ms;     /* first to last kernel of the call                */
    uint64_t units;          /* 64 x 64 work units the sweep processed          */
    uint32_t dense_primes;   /* K used                                          */
    uint32_t workgroups;     /* grid used                                       */
    uint32_t graph;          /* 0 launched call by call, 1 replayed a captured  */
                             /* graph, 2 captured a new graph and launched it   */
    uint32_t reserved;
} cuboid_timing;

/* Turn per-call HIP-event timing on (1) or off (0). */
int cuboid_enable_timing(cuboid_ctx *ctx, int on);
/* Batched and plain sieve calls over rows below 2^24 run as one replay of a
 * captured HIP graph (1, the default) or as separate launches (0).  Either
 * way the results are the same.  A graph is captured on first use of a
 * request count, prime list, tuning and buffer set, and replayed for later
 * calls that share them; up to 8 graphs are kept per context.  Turning graphs
 * off frees them.  E_DEVICE if capture fails. */
int cuboid_enable_graphs(cuboid_ctx *ctx, int on);
/* Timing of the last sieve call on this context. */
int cuboid_last_timing(cuboid_ctx *ctx, cuboid_timing *out);

#ifdef __cplusplus
}
#endif

#endif /* CUBOID_H */
