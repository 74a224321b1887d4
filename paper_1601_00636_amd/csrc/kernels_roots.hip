// Integer-root candidates for sieve survivors and their evaluation modulo three
// 62-bit primes.  Q_pq(t) of eq. (1.1) of arXiv:1601.00636 is a monic
// polynomial in s = t^2 with constant term -p^10 q^10, so an integer root has
// t^2 | p^10 q^10, i.e. t | p^5 q^5 (on the axes q = 0 or p = 0 the lowest
// non-zero coefficient is p^8 or q^8, and t | p^4 or q^4).  A root bound on s
// (Fujiwara's) limits the divisors tried; a candidate that vanishes modulo all
// three primes is passed to the exact CPU check.  p, q < 2^32, so the bound
// on t reaches about 2^66.5 (at p = q = 2^32 - 1): candidates are 128-bit.
#include "devmath.h"
#include "internal.h"

namespace cuboid {

namespace {

typedef unsigned __int128 u128;

constexpr uint64_t kMask62 = (1ull << 62) - 1;
__constant__ uint64_t kModC[3] = {57, 87, 117};   // moduli 2^62 - c

// a * b mod M for M = 2^62 - c, c < 128, a, b < M
__device__ __forceinline__ uint64_t mulmod62(uint64_t a, uint64_t b, uint64_t c, uint64_t M) {
    const uint64_t lo = a * b, hi = __umul64hi(a, b);      // product < 2^124
    const uint64_t H = (hi << 2) | (lo >> 62), L = lo & kMask62;
    // H * 2^62 + L == H * c + L  (mod M)
    const uint64_t l2 = H * c, h2 = __umul64hi(H, c);
    const uint64_t G = (h2 << 2) | (l2 >> 62);
    uint64_t y = G * c + (l2 & kMask62) + L;
    while (y >= M) y -= M;
    return y;
}

__device__ __forceinline__ uint64_t addmod62(uint64_t a, uint64_t b, uint64_t M) {
    const uint64_t s = a + b;
    return s >= M ? s - M : s;
}

__device__ __forceinline__ uint64_t submod62(uint64_t a, uint64_t b, uint64_t M) {
    return a >= b ? a - b : a + (M - b);
}

__device__ __forceinline__ uint64_t small_mul(uint64_t a, uint32_t k, uint64_t c, uint64_t M) {
    return mulmod62(a, k, c, M);
}

// x mod M for any 64-bit x: x < 2^64 = 4 M + 4 c, so at most four subtractions
__device__ __forceinline__ uint64_t red64(uint64_t x, uint64_t M) {
    while (x >= M) x -= M;
    return x;
}

// Q_pq(t) mod M for t = t_hi 2^64 + t_lo, coefficients as in eq. (1.1)
__device__ uint64_t q_mod62(uint32_t p, uint32_t q, uint64_t t_lo, uint64_t t_hi, uint64_t c) {
    const uint64_t M = (1ull << 62) - c;
    const uint64_t P = red64((uint64_t)p * p, M), Q = red64((uint64_t)q * q, M);   // p^2 < 2^64
    // 2^64 = 4 M + 4 c, so t = t_hi (4 c) + t_lo (mod M)
    const uint64_t t = addmod62(mulmod62(red64(t_hi, M), 4 * c, c, M), red64(t_lo, M), M);
    const uint64_t s = mulmod62(t, t, c, M);
    const uint64_t P2 = mulmod62(P, P, c, M), Q2 = mulmod62(Q, Q, c, M);
    const uint64_t P3 = mulmod62(P2, P, c, M), Q3 = mulmod62(Q2, Q, c, M);
    const uint64_t P4 = mulmod62(P2, P2, c, M), Q4 = mulmod62(Q2, Q2, c, M);
    const uint64_t P5 = mulmod62(P4, P, c, M), Q5 = mulmod62(Q4, Q, c, M);
    const uint64_t PQ3 = mulmod62(P, Q3, c, M), P2Q2 = mulmod62(P2, Q2, c, M);
    const uint64_t P3Q = mulmod62(P3, Q, c, M);
    // s^4: (2Q + P)(3Q - 2P)
    const uint64_t c8 = mulmod62(addmod62(small_mul(Q, 2, c, M), P, M),
                                 submod62(small_mul(Q, 3, c, M), small_mul(P, 2, c, M), M), c, M);
    // s^3: Q^4 + 10 P Q^3 + 4 P^2 Q^2 - 14 P^3 Q + P^4
    uint64_t c6 = addmod62(Q4, small_mul(PQ3, 10, c, M), M);
    c6 = addmod62(c6, small_mul(P2Q2, 4, c, M), M);
    c6 = submod62(c6, small_mul(P3Q, 14, c, M), M);
    c6 = addmod62(c6, P4, M);
    // s^2: -P Q (Q^4 - 14 P Q^3 + 4 P^2 Q^2 + 10 P^3 Q + P^4)
    uint64_t in4 = submod62(Q4, small_mul(PQ3, 14, c, M), M);
    in4 = addmod62(in4, small_mul(P2Q2, 4, c, M), M);
    in4 = addmod62(in4, small_mul(P3Q, 10, c, M), M);
    in4 = addmod62(in4, P4, M);
    const uint64_t c4 = submod62(0, mulmod62(mulmod62(P, Q, c, M), in4, c, M), M);
    // s^1: -P^3 Q^3 (Q + 2P)(3P - 2Q)
    const uint64_t a2 = addmod62(Q, small_mul(P, 2, c, M), M);
    const uint64_t b2 = submod62(small_mul(P, 3, c, M), small_mul(Q, 2, c, M), M);
    const uint64_t c2 = submod62(0, mulmod62(mulmod62(P3, Q3, c, M), mulmod62(a2, b2, c, M), c, M), M);
    // s^0: -P^5 Q^5
    const uint64_t c0 = submod62(0, mulmod62(P5, Q5, c, M), M);
    uint64_t v = addmod62(s, c8, M);
    v = addmod62(mulmod62(v, s, c, M), c6, M);
    v = addmod62(mulmod62(v, s, c, M), c4, M);
    v = addmod62(mulmod62(v, s, c, M), c2, M);
    v = addmod62(mulmod62(v, s, c, M), c0, M);
    return v;
}

// Trial division of x by the primes below 2^16; appends (prime, exponent*mult)
// to the candidate's factor list, merging with primes already present.
__device__ void add_factors(uint32_t x, uint32_t mult, const uint32_t *primes16,
                            const uint32_t *magic16, uint32_t n16, RootCand &c) {
    for (uint32_t i = 0; i < n16 && x > 1; ++i) {
        const uint32_t l = primes16[i];
        if ((uint64_t)l * l > x) break;
        uint32_t rem;
        uint32_t qt = divr(x, l, magic16[i], &rem);
        if (rem) continue;
        uint32_t e = 0;
        do { x = qt; ++e; qt = divr(x, l, magic16[i], &rem); } while (rem == 0);
        uint32_t k = 0;
        while (k < c.nf && c.fp[k] != l) ++k;
        if (k == c.nf) { c.fp[k] = l; c.fe[k] = 0; ++c.nf; }
        c.fe[k] += e * mult;
    }
    if (x > 1) {
        uint32_t k = 0;
        while (k < c.nf && c.fp[k] != x) ++k;
        if (k == c.nf) { c.fp[k] = x; c.fe[k] = 0; ++c.nf; }
        c.fe[k] += mult;
    }
}

__global__ void root_factor_kernel(const uint32_t *pp, const uint32_t *qq, uint64_t n,
                                   const uint32_t *primes16, const uint32_t *magic16, uint32_t n16,
                                   RootCand *out) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        RootCand c;
        c.p = pp[i];
        c.q = qq[i];
        c.nf = 0;
        c.pad = 0;
        for (int k = 0; k < 20; ++k) { c.fp[k] = 0; c.fe[k] = 0; }
        c.bound_lo = c.bound_hi = 0;
        c.ndiv = 0;
        if (c.p == 0 && c.q == 0) { out[i] = c; continue; }     // Q = t^10: no t > 0
        if (c.q == 0) add_factors(c.p, 4, primes16, magic16, n16, c);
        else if (c.p == 0) add_factors(c.q, 4, primes16, magic16, n16, c);
        else {
            add_factors(c.p, 5, primes16, magic16, n16, c);
            add_factors(c.q, 5, primes16, magic16, n16, c);
        }
        uint64_t nd = 1;
        for (uint32_t k = 0; k < c.nf; ++k) {
            const uint64_t e1 = c.fe[k] + 1;
            nd = (nd > (1ull << 62) / e1) ? (1ull << 62) : nd * e1;
        }
        c.ndiv = nd;
        // Root bound: upper bounds of |coefficient| from the terms of eq. (1.1)
        // taken with plus signs, then Fujiwara: every root s of the monic
        // quintic has |s| <= 2 max(|a4|, |a3|^1/2, |a2|^1/3, |a1|^1/4, |a0/2|^1/5).
        const double P = (double)c.p * c.p, Q = (double)c.q * c.q;
        const double a4 = (2 * Q + P) * (3 * Q + 2 * P);
        const double a3 = Q * Q * Q * Q + 10 * P * Q * Q * Q + 4 * P * P * Q * Q + 14 * P * P * P * Q +
                          P * P * P * P;
        const double a2 = P * Q * (Q * Q * Q * Q + 14 * P * Q * Q * Q + 4 * P * P * Q * Q +
                                   10 * P * P * P * Q + P * P * P * P);
        const double a1 = P * P * P * Q * Q * Q * (Q + 2 * P) * (3 * P + 2 * Q);
        const double a0 = P * P * P * P * P * Q * Q * Q * Q * Q;
        double m = a4;
        m = fmax(m, sqrt(a3));
        m = fmax(m, cbrt(a2));
        m = fmax(m, sqrt(sqrt(a1)));
        m = fmax(m, pow(a0 / 2, 0.2));
        const double tb = sqrt(2 * m) * (1.0 + 1e-9) + 2.0;
        // tb < 2^67: its high and low 64-bit halves (both exact in double)
        const double two64 = 18446744073709551616.0;
        const double hi = floor(tb / two64);
        const double lo = tb - hi * two64;
        c.bound_hi = (uint64_t)hi;
        c.bound_lo = lo >= 18446744073709549568.0 ? ~0ull : (uint64_t)lo;
        out[i] = c;
    }
}

__global__ void root_eval_kernel(const RootCand *cand, uint64_t n_cand, const uint64_t *prefix,
                                 uint64_t w0, uint64_t nwork, RootHit *hits, uint64_t cap,
                                 unsigned long long *n_hits) {
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < nwork;
         g += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t w = w0 + g;
        // candidate index: last i with prefix[i] <= w
        uint64_t lo = 0, hi = n_cand;
        while (hi - lo > 1) {
            const uint64_t mid = (lo + hi) >> 1;
            if (prefix[mid] <= w) lo = mid; else hi = mid;
        }
        const RootCand &c = cand[lo];
        uint64_t k = w - prefix[lo];
        const u128 bound = (u128)c.bound_hi << 64 | c.bound_lo;
        // mixed-radix digits of k give the exponent of each prime in t; t stays
        // at most bound < 2^68 before each step, so t * fp < 2^100 cannot wrap
        u128 t = 1;
        bool over = false;
        for (uint32_t f = 0; f < c.nf && !over; ++f) {
            const uint64_t e1 = c.fe[f] + 1;
            uint64_t d = k % e1;
            k /= e1;
            while (d--) {
                t *= c.fp[f];
                if (t > bound) { over = true; break; }
            }
        }
        if (over) continue;
        const uint64_t t_lo = (uint64_t)t, t_hi = (uint64_t)(t >> 64);
        bool zero = true;
        for (int j = 0; j < 3 && zero; ++j) zero = q_mod62(c.p, c.q, t_lo, t_hi, kModC[j]) == 0;
        if (zero) {
            const unsigned long long pos = atomicAdd(n_hits, 1ull);
            if (pos < cap) {
                RootHit h;
                h.cand = (uint32_t)lo;
                h.pad = 0;
                h.t_lo = t_lo;
                h.t_hi = t_hi;
                hits[pos] = h;
            }
        }
    }
}

}  // namespace

hipError_t launch_root_factor(const uint32_t *p, const uint32_t *q, uint64_t n,
                              const uint32_t *primes16, const uint32_t *magic16, uint32_t n16,
                              RootCand *out, hipStream_t s) {
    if (!n) return hipSuccess;
    uint64_t g = (n + 63) / 64;
    if (g > 65535) g = 65535;
    hipLaunchKernelGGL(root_factor_kernel, dim3((unsigned)g), dim3(64), 0, s, p, q, n, primes16,
                       magic16, n16, out);
    return hipGetLastError();
}

hipError_t launch_root_eval(const RootCand *c, uint64_t n_cand, const uint64_t *prefix,
                            uint64_t w0, uint64_t nwork, RootHit *hits, uint64_t cap,
                            unsigned long long *n_hits, hipStream_t s) {
    if (!nwork) return hipSuccess;
    uint64_t g = (nwork + 255) / 256;
    if (g > (1u << 20)) g = 1u << 20;
    hipLaunchKernelGGL(root_eval_kernel, dim3((unsigned)g), dim3(256), 0, s, c, n_cand, prefix, w0,
                       nwork, hits, cap, n_hits);
    return hipGetLastError();
}

}  // namespace cuboid
