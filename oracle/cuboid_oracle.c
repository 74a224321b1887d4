/*
 * ORACLE — test infrastructure only.
 *
 * A plain, slow, obviously correct CPU definition of what the modulo-primes
 * cuboid sieve computes.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this code; the product library never
 * links, loads or calls it, and the two share no source.
 *
 * Paper: R.R. Gallyamov, I.R. Kadyrov, D.D. Kashelevskiy, N.G. Kutlugallyamov,
 * R.A. Sharipov, "A fast modulo primes algorithm for searching perfect cuboids
 * and its implementation" (arXiv:1601.00636).
 *
 * What each function follows:
 *   oracle_coeffs_mod_r / oracle_q_mod_r  eq. (1.1) reduced modulo r, eq. (2.2)
 *   oracle_table                          Definition 1.1 and eq. (2.3)
 *   oracle_u_entry                        one entry of Definition 1.1, for
 *                                         primes whose whole table is too
 *                                         large to build
 *   oracle_pack                           the byte packing of eq. (2.6)
 *   oracle_sieve                          section 2 (the bit sieve) restricted to
 *                                         the domain of Conjecture 1.1
 *   oracle_sieve_region                   the same over region (1.2), section 5
 *
 * Integer arithmetic throughout; no floating point.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* residue of x*y modulo r for residues x,y < r < 2^32 */
static uint64_t mul_r(uint64_t x, uint64_t y, uint64_t r) { return (x * y) % r; }

/* (r - x) mod r: the residue of -x */
static uint64_t neg_r(uint64_t x, uint64_t r) { return x == 0 ? 0 : r - x; }

/*
 * The six coefficients of Q_pq(t) (eq. 1.1) modulo r, in ascending powers of
 * t: out[0] is the constant term, out[k] multiplies t^(2k), out[5] = 1.
 *   t^10 : 1
 *   t^8  : (2 q^2 + p^2)(3 q^2 - 2 p^2)
 *   t^6  : q^8 + 10 p^2 q^6 + 4 p^4 q^4 - 14 p^6 q^2 + p^8
 *   t^4  : -p^2 q^2 (q^8 - 14 p^2 q^6 + 4 p^4 q^4 + 10 p^6 q^2 + p^8)
 *   t^2  : -p^6 q^6 (q^2 + 2 p^2)(3 p^2 - 2 q^2)
 *   t^0  : -q^10 p^10
 */
void oracle_coeffs_mod_r(uint64_t p, uint64_t q, uint32_t r, uint32_t out[6])
{
    uint64_t R = r;
    uint64_t p1 = p % R, q1 = q % R;
    uint64_t p2 = mul_r(p1, p1, R), q2 = mul_r(q1, q1, R);
    uint64_t p4 = mul_r(p2, p2, R), q4 = mul_r(q2, q2, R);
    uint64_t p6 = mul_r(p4, p2, R), q6 = mul_r(q4, q2, R);
    uint64_t p8 = mul_r(p4, p4, R), q8 = mul_r(q4, q4, R);
    uint64_t p10 = mul_r(p8, p2, R), q10 = mul_r(q8, q2, R);

    /* t^8 */
    uint64_t a8 = (2 * q2 + p2) % R;
    uint64_t b8 = (3 * q2 + neg_r((2 * p2) % R, R)) % R;
    uint64_t c8 = mul_r(a8, b8, R);

    /* t^6 */
    uint64_t c6 = (q8
                   + 10 * mul_r(p2, q6, R)
                   + 4 * mul_r(p4, q4, R)
                   + neg_r((14 * mul_r(p6, q2, R)) % R, R)
                   + p8) % R;

    /* t^4 */
    uint64_t in4 = (q8
                    + neg_r((14 * mul_r(p2, q6, R)) % R, R)
                    + 4 * mul_r(p4, q4, R)
                    + 10 * mul_r(p6, q2, R)
                    + p8) % R;
    uint64_t c4 = neg_r(mul_r(mul_r(p2, q2, R), in4, R), R);

    /* t^2 */
    uint64_t a2 = (q2 + 2 * p2) % R;
    uint64_t b2 = (3 * p2 + neg_r((2 * q2) % R, R)) % R;
    uint64_t c2 = neg_r(mul_r(mul_r(mul_r(p6, q6, R), a2, R), b2, R), R);

    /* t^0 */
    uint64_t c0 = neg_r(mul_r(q10, p10, R), R);

    out[0] = (uint32_t)c0;
    out[1] = (uint32_t)c2;
    out[2] = (uint32_t)c4;
    out[3] = (uint32_t)c6;
    out[4] = (uint32_t)c8;
    out[5] = (uint32_t)(1 % R);
}

/* Q_pq(t) mod r (eq. 2.2): the sum of c_k t^(2k) over the six terms. */
uint32_t oracle_q_mod_r(uint64_t p, uint64_t q, uint64_t t, uint32_t r)
{
    uint32_t c[6];
    uint64_t R = r;
    oracle_coeffs_mod_r(p, q, r, c);
    uint64_t t1 = t % R;
    uint64_t t2 = mul_r(t1, t1, R);
    uint64_t pw = 1, acc = 0;
    for (int k = 0; k < 6; ++k) {
        acc = (acc + mul_r(c[k], pw, R)) % R;
        pw = mul_r(pw, t2, R);
    }
    return (uint32_t)acc;
}

/*
 * Unsolvability table of Definition 1.1 / eq. (2.3):
 *   u[a*r + b] = 1  iff  no t in [0, r) has Q_ab(t) = 0 mod r,
 * for 0 <= a, b < r (a is the row p~, b the column q~).  Every t is tried
 * directly; the powers t^(2k) mod r are tabulated once per t.
 * Requires r < 2^16 so that c_k * t^(2k) stays below 2^32 and their sum of
 * six fits comfortably in 64 bits.
 */
int oracle_table(uint32_t r, uint8_t *u)
{
    if (r < 2 || r >= 65536) return -1;
    uint64_t R = r;
    uint32_t *pw = (uint32_t *)malloc(sizeof(uint32_t) * 6 * (size_t)r);
    if (!pw) return -2;
    for (uint64_t t = 0; t < R; ++t) {
        uint64_t t2 = mul_r(t, t, R), x = 1 % R;
        for (int k = 0; k < 6; ++k) { pw[k * (size_t)r + t] = (uint32_t)x; x = mul_r(x, t2, R); }
    }
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t a = 0; a < (int64_t)r; ++a) {
        for (uint64_t b = 0; b < R; ++b) {
            uint32_t c[6];
            oracle_coeffs_mod_r((uint64_t)a, b, r, c);
            int solvable = 0;
            for (uint64_t t = 0; t < R && !solvable; ++t) {
                uint64_t s = 0;
                for (int k = 0; k < 6; ++k) s += (uint64_t)c[k] * pw[k * (size_t)r + t];
                if (s % R == 0) solvable = 1;
            }
            u[(size_t)a * r + b] = (uint8_t)!solvable;
        }
    }
    free(pw);
    return 0;
}

/*
 * Byte packing of eq. (2.6): the r*r bits in row-major order (linear index
 * a*r + b), eight to a byte, least significant bit first (the paper prints each
 * byte with its highest bit on the left), the last byte zero-padded.
 * Returns the number of bytes, ceil(r*r / 8).
 */
uint64_t oracle_pack(uint32_t r, const uint8_t *u, uint8_t *out)
{
    uint64_t nbits = (uint64_t)r * r, nbytes = (nbits + 7) / 8;
    memset(out, 0, nbytes);
    for (uint64_t i = 0; i < nbits; ++i)
        if (u[i]) out[i / 8] |= (uint8_t)(1u << (i % 8));
    return nbytes;
}

/*
 * u_r(a, b) for one entry, from Definition 1.1: 1 iff no t in [0, r) has
 * Q_ab(t) = 0 mod r.  r evaluations of oracle_q_mod_r.
 */
int oracle_u_entry(uint32_t a, uint32_t b, uint32_t r)
{
    for (uint64_t t = 0; t < r; ++t)
        if (oracle_q_mod_r(a, b, t, r) == 0) return 0;
    return 1;
}

/* greatest common divisor, Euclid */
static uint64_t gcd_u64(uint64_t a, uint64_t b)
{
    while (b) { uint64_t t = a % b; a = b; b = t; }
    return a;
}

static int cmp_u64(const void *x, const void *y)
{
    uint64_t a = *(const uint64_t *)x, b = *(const uint64_t *)y;
    return (a > b) - (a < b);
}

/*
 * The sieve over the rectangle p0..p1 x q0..q1 (inclusive).
 *
 * Domain (Conjecture 1.1): pairs with p != q and gcd(p, q) = 1; their number is
 * *n_pairs.  Each such pair is tested against the tables of `primes` (which the
 * caller passes in ascending order, with their unpacked tables `tables[i]`,
 * r_i*r_i bytes each) in that order; the first prime whose unsolvability bit
 * u_r(p mod r, q mod r) is 1 rejects the pair and counts[i] is incremented.
 * With tables == NULL every bit the walk needs is evaluated by oracle_u_entry
 * instead (prime lists whose tables are too large to build).  A
 * pair no prime rejects is a survivor, reported as the index
 * (p - p0) * (q1 - q0 + 1) + (q - q0); survivors come back ascending.
 *
 * Up to `cap` survivors are stored; *n_surv receives the total.
 * Rows are split across `nthreads` OpenMP threads (0 = runtime default).
 */
int oracle_sieve(uint32_t p0, uint32_t p1, uint32_t q0, uint32_t q1,
                 const uint32_t *primes, uint32_t n_primes,
                 const uint8_t *const *tables,
                 uint64_t *counts, uint64_t *n_pairs,
                 uint64_t *surv, uint64_t cap, uint64_t *n_surv,
                 int nthreads)
{
    if (p0 > p1 || q0 > q1) return -1;
    uint64_t width = (uint64_t)q1 - q0 + 1;
    uint64_t total_pairs = 0, total_surv = 0;
    memset(counts, 0, sizeof(uint64_t) * n_primes);
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif
    uint64_t *tc = (uint64_t *)calloc((size_t)nthreads * (n_primes + 1), sizeof(uint64_t));
    uint64_t **ts = (uint64_t **)calloc((size_t)nthreads, sizeof(uint64_t *));
    uint64_t *tn = (uint64_t *)calloc((size_t)nthreads, sizeof(uint64_t));
    uint64_t *tcap = (uint64_t *)calloc((size_t)nthreads, sizeof(uint64_t));
    if (!tc || !ts || !tn || !tcap) return -2;

    #pragma omp parallel num_threads(nthreads)
    {
#ifdef _OPENMP
        int tid = omp_get_thread_num();
#else
        int tid = 0;
#endif
        uint64_t *cnt = tc + (size_t)tid * (n_primes + 1);
        #pragma omp for schedule(dynamic, 16)
        for (int64_t pp = (int64_t)p0; pp <= (int64_t)p1; ++pp) {
            uint64_t p = (uint64_t)pp;
            for (uint64_t q = q0; q <= q1; ++q) {
                if (p == q) continue;
                if (gcd_u64(p, q) != 1) continue;
                cnt[n_primes] += 1;
                int rejected = 0;
                for (uint32_t i = 0; i < n_primes; ++i) {
                    uint64_t r = primes[i];
                    const int u = tables ? tables[i][(p % r) * r + (q % r)]
                                         : oracle_u_entry((uint32_t)(p % r), (uint32_t)(q % r), (uint32_t)r);
                    if (u) { cnt[i] += 1; rejected = 1; break; }
                }
                if (!rejected) {
                    if (tn[tid] == tcap[tid]) {
                        tcap[tid] = tcap[tid] ? 2 * tcap[tid] : 64;
                        ts[tid] = (uint64_t *)realloc(ts[tid], sizeof(uint64_t) * tcap[tid]);
                    }
                    ts[tid][tn[tid]++] = (p - p0) * width + (q - q0);
                }
            }
        }
    }
    for (int t = 0; t < nthreads; ++t) {
        for (uint32_t i = 0; i < n_primes; ++i) counts[i] += tc[(size_t)t * (n_primes + 1) + i];
        total_pairs += tc[(size_t)t * (n_primes + 1) + n_primes];
        total_surv += tn[t];
    }
    uint64_t *all = (uint64_t *)malloc(sizeof(uint64_t) * (total_surv ? total_surv : 1));
    uint64_t k = 0;
    for (int t = 0; t < nthreads; ++t) {
        if (tn[t]) memcpy(all + k, ts[t], sizeof(uint64_t) * tn[t]);
        k += tn[t];
        free(ts[t]);
    }
    qsort(all, total_surv, sizeof(uint64_t), cmp_u64);
    for (uint64_t i = 0; i < total_surv && i < cap; ++i) surv[i] = all[i];
    *n_surv = total_surv;
    *n_pairs = total_pairs;
    free(all); free(tc); free(ts); free(tn); free(tcap);
    return 0;
}

/*
 * Smallest integer q >= 1 allowed by the lower bound of region (1.2),
 * min(cbrt(p/9), p/59) <= q, in exact integers: the smaller of the least q
 * with 9 q^3 >= p and the least q with 59 q >= p.
 */
uint64_t oracle_region_qmin(uint64_t p)
{
    uint64_t a = 1;
    while (9 * a * a * a < p) ++a;
    uint64_t b = (p + 58) / 59;
    if (b < 1) b = 1;
    return a < b ? a : b;
}

/*
 * The sieve over region (1.2) for p0 <= p <= p1: for each p every integer q
 * with oracle_region_qmin(p) <= q <= 59 p, in the domain of Conjecture 1.1.
 * counts/n_pairs as in oracle_sieve; survivors are returned as (p, q) pairs
 * (surv_pq[2k], surv_pq[2k+1]) in ascending (p, q) order.  *max_depth gets the
 * largest index i (1-based, into `primes`) of a first rejecting prime seen.
 */
int oracle_sieve_region(uint32_t p0, uint32_t p1,
                        const uint32_t *primes, uint32_t n_primes,
                        const uint8_t *const *tables,
                        uint64_t *counts, uint64_t *n_pairs,
                        uint64_t *surv_pq, uint64_t cap, uint64_t *n_surv,
                        uint32_t *max_depth, int nthreads)
{
    if (p0 < 1 || p0 > p1) return -1;
    uint64_t *row_n = (uint64_t *)calloc((size_t)(p1 - p0 + 1), sizeof(uint64_t));
    uint64_t *tc;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif
    tc = (uint64_t *)calloc((size_t)nthreads * (n_primes + 2), sizeof(uint64_t));
    if (!row_n || !tc) return -2;
    uint64_t found = 0;
    memset(counts, 0, sizeof(uint64_t) * n_primes);
    #pragma omp parallel num_threads(nthreads)
    {
#ifdef _OPENMP
        int tid = omp_get_thread_num();
#else
        int tid = 0;
#endif
        uint64_t *cnt = tc + (size_t)tid * (n_primes + 2);
        #pragma omp for schedule(dynamic, 16)
        for (int64_t pp = (int64_t)p0; pp <= (int64_t)p1; ++pp) {
            uint64_t p = (uint64_t)pp;
            uint64_t qlo = oracle_region_qmin(p), qhi = 59 * p;
            for (uint64_t q = qlo; q <= qhi; ++q) {
                if (p == q || gcd_u64(p, q) != 1) continue;
                cnt[n_primes] += 1;
                int rejected = 0;
                for (uint32_t i = 0; i < n_primes; ++i) {
                    uint64_t r = primes[i];
                    if (tables[i][(p % r) * r + (q % r)]) {
                        cnt[i] += 1;
                        if (i + 1 > cnt[n_primes + 1]) cnt[n_primes + 1] = i + 1;
                        rejected = 1;
                        break;
                    }
                }
                if (!rejected) row_n[p - p0] += 1;
            }
        }
    }
    uint32_t depth = 0;
    uint64_t pairs = 0;
    for (int t = 0; t < nthreads; ++t) {
        for (uint32_t i = 0; i < n_primes; ++i) counts[i] += tc[(size_t)t * (n_primes + 2) + i];
        pairs += tc[(size_t)t * (n_primes + 2) + n_primes];
        if (tc[(size_t)t * (n_primes + 2) + n_primes + 1] > depth)
            depth = (uint32_t)tc[(size_t)t * (n_primes + 2) + n_primes + 1];
    }
    /* second, serial pass over rows that hold survivors, to list them in order */
    for (uint64_t p = p0; p <= p1; ++p) {
        if (!row_n[p - p0]) continue;
        uint64_t qlo = oracle_region_qmin(p), qhi = 59 * p;
        for (uint64_t q = qlo; q <= qhi; ++q) {
            if (p == q || gcd_u64(p, q) != 1) continue;
            int rejected = 0;
            for (uint32_t i = 0; i < n_primes && !rejected; ++i) {
                uint64_t r = primes[i];
                if (tables[i][(p % r) * r + (q % r)]) rejected = 1;
            }
            if (!rejected) {
                if (found < cap) { surv_pq[2 * found] = p; surv_pq[2 * found + 1] = q; }
                ++found;
            }
        }
    }
    *n_surv = found;
    *n_pairs = pairs;
    *max_depth = depth;
    free(row_n); free(tc);
    return 0;
}
