// Device arithmetic shared by the libcuboid kernels: residues modulo a 16-bit
// modulus by multiply-high, and Q_pq(t) mod r (eq. 1.1 of arXiv:1601.00636).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cuboid {

// x mod r for any x < 2^32 and 2 <= r < 2^32, with m = floor(2^32 / r).
// umulhi(x, m) is floor(x / r) or one less, so one correction suffices.
__device__ __forceinline__ uint32_t modr(uint32_t x, uint32_t r, uint32_t m) {
    uint32_t qe = __umulhi(x, m);
    uint32_t t = x - qe * r;
    return t >= r ? t - r : t;
}

// quotient and remainder of x by r, same contract as modr
__device__ __forceinline__ uint32_t divr(uint32_t x, uint32_t r, uint32_t m, uint32_t *rem) {
    uint32_t qe = __umulhi(x, m);
    uint32_t t = x - qe * r;
    if (t >= r) { t -= r; ++qe; }
    *rem = t;
    return qe;
}

// product of two residues of a modulus r < 2^16
__device__ __forceinline__ uint32_t mulr(uint32_t a, uint32_t b, uint32_t r, uint32_t m) {
    return modr(a * b, r, m);
}

__device__ __forceinline__ uint32_t negr(uint32_t a, uint32_t r) { return a ? r - a : 0u; }

// Coefficients of Q_pq as a polynomial in s = t^2, modulo r < 2^16, for
// residues pr = p mod r, qr = q mod r.  With P = p^2, Q = q^2 (eq. 1.1):
//   s^4: (2Q + P)(3Q - 2P)
//   s^3: Q^4 + 10 P Q^3 + 4 P^2 Q^2 - 14 P^3 Q + P^4
//   s^2: -P Q (Q^4 - 14 P Q^3 + 4 P^2 Q^2 + 10 P^3 Q + P^4)
//   s^1: -P^3 Q^3 (Q + 2P)(3P - 2Q)
//   s^0: -P^5 Q^5
struct QCoef {
    uint32_t c8, c6, c4, c2, c0;
};

__device__ __forceinline__ QCoef q_coeffs(uint32_t pr, uint32_t qr, uint32_t r, uint32_t m) {
    const uint32_t P = mulr(pr, pr, r, m), Q = mulr(qr, qr, r, m);
    const uint32_t P2 = mulr(P, P, r, m), Q2 = mulr(Q, Q, r, m);
    const uint32_t P3 = mulr(P2, P, r, m), Q3 = mulr(Q2, Q, r, m);
    const uint32_t P4 = mulr(P2, P2, r, m), Q4 = mulr(Q2, Q2, r, m);
    const uint32_t P5 = mulr(P4, P, r, m), Q5 = mulr(Q4, Q, r, m);
    const uint32_t PQ3 = mulr(P, Q3, r, m), P2Q2 = mulr(P2, Q2, r, m), P3Q = mulr(P3, Q, r, m);
    QCoef c;
    // every sum below stays under 30 r < 2^21
    c.c8 = mulr(modr(2 * Q + P, r, m), modr(3 * Q + 2 * (r - P), r, m), r, m);
    c.c6 = modr(Q4 + 10 * PQ3 + 4 * P2Q2 + 14 * (r - P3Q) + P4, r, m);
    const uint32_t in4 = modr(Q4 + 14 * (r - PQ3) + 4 * P2Q2 + 10 * P3Q + P4, r, m);
    c.c4 = negr(mulr(mulr(P, Q, r, m), in4, r, m), r);
    const uint32_t a2 = modr(Q + 2 * P, r, m), b2 = modr(3 * P + 2 * (r - Q), r, m);
    c.c2 = negr(mulr(mulr(P3, Q3, r, m), mulr(a2, b2, r, m), r, m), r);
    c.c0 = negr(mulr(P5, Q5, r, m), r);
    return c;
}

// Horner in s: ((((s + c8) s + c6) s + c4) s + c2) s + c0, modulo r
__device__ __forceinline__ uint32_t q_eval_s(const QCoef &c, uint32_t s, uint32_t r, uint32_t m) {
    uint32_t v = s + c.c8;
    v = v >= r ? v - r : v;
    v = mulr(v, s, r, m) + c.c6;
    v = v >= r ? v - r : v;
    v = mulr(v, s, r, m) + c.c4;
    v = v >= r ? v - r : v;
    v = mulr(v, s, r, m) + c.c2;
    v = v >= r ? v - r : v;
    v = mulr(v, s, r, m) + c.c0;
    v = v >= r ? v - r : v;
    return v;
}

// first index i in [0, n) with prefix[i + 1] > g (prefix[0] = 0, ascending)
__device__ __forceinline__ uint32_t find_segment(const uint64_t *prefix, uint32_t n, uint64_t g) {
    uint32_t lo = 0, hi = n;   // answer in [lo, hi)
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

}  // namespace cuboid
