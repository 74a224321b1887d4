// Exact confirmation of integer roots on the CPU: Q_pq(t) of eq. (1.1) of
// arXiv:1601.00636 evaluated in fixed-width signed multiprecision arithmetic,
// and the four inequalities of Theorem 1.1.  p, q < 2^32 and t < 2^70 keep
// every intermediate below 2^720 (s^5 = t^10 < 2^700, P^5 Q^5 < 2^640), well
// inside the 1024-bit width; larger t is reported as an overflow.
#include "bigint.h"

#include <string.h>

#include <algorithm>
#include <string>

namespace cuboid {

namespace {

constexpr int kLimbs = 16;   // 1024 bits
typedef unsigned __int128 u128;

struct Big {
    bool neg = false;
    uint64_t l[kLimbs] = {0};

    static Big from_u64(uint64_t v) {
        Big b;
        b.l[0] = v;
        return b;
    }
    static Big from_i128(bool negative, u128 mag) {
        Big b;
        b.l[0] = (uint64_t)mag;
        b.l[1] = (uint64_t)(mag >> 64);
        b.neg = negative && (mag != 0);
        return b;
    }
    bool is_zero() const {
        for (int i = 0; i < kLimbs; ++i)
            if (l[i]) return false;
        return true;
    }
};

// |a| compared with |b|
int cmp_mag(const Big &a, const Big &b) {
    for (int i = kLimbs - 1; i >= 0; --i) {
        if (a.l[i] != b.l[i]) return a.l[i] < b.l[i] ? -1 : 1;
    }
    return 0;
}

// |a| + |b| into r (magnitude only); returns false on overflow
bool add_mag(const Big &a, const Big &b, Big &r) {
    u128 carry = 0;
    for (int i = 0; i < kLimbs; ++i) {
        u128 s = (u128)a.l[i] + b.l[i] + carry;
        r.l[i] = (uint64_t)s;
        carry = s >> 64;
    }
    return carry == 0;
}

// |a| - |b| into r, requires |a| >= |b|
void sub_mag(const Big &a, const Big &b, Big &r) {
    uint64_t borrow = 0;
    for (int i = 0; i < kLimbs; ++i) {
        u128 d = (u128)a.l[i] - b.l[i] - borrow;
        r.l[i] = (uint64_t)d;
        borrow = (uint64_t)(d >> 64) ? 1 : 0;
    }
}

bool add(const Big &a, const Big &b, Big &r) {
    Big out;
    if (a.neg == b.neg) {
        if (!add_mag(a, b, out)) return false;
        out.neg = a.neg;
    } else if (cmp_mag(a, b) >= 0) {
        sub_mag(a, b, out);
        out.neg = a.neg;
    } else {
        sub_mag(b, a, out);
        out.neg = b.neg;
    }
    if (out.is_zero()) out.neg = false;
    r = out;
    return true;
}

Big negate(Big a) {
    if (!a.is_zero()) a.neg = !a.neg;
    return a;
}

bool mul(const Big &a, const Big &b, Big &r) {
    Big out;
    for (int i = 0; i < kLimbs; ++i) {
        if (!a.l[i]) continue;
        u128 carry = 0;
        for (int j = 0; j < kLimbs; ++j) {
            if (i + j >= kLimbs) {
                if (b.l[j] || carry) return false;
                continue;
            }
            u128 cur = (u128)a.l[i] * b.l[j] + out.l[i + j] + carry;
            out.l[i + j] = (uint64_t)cur;
            carry = cur >> 64;
        }
        if (carry) return false;
    }
    out.neg = (a.neg != b.neg) && !out.is_zero();
    r = out;
    return true;
}

struct Ctx {
    bool ok = true;
    Big mul(const Big &a, const Big &b) {
        Big r;
        if (!cuboid::mul(a, b, r)) ok = false;
        return r;
    }
    Big add(const Big &a, const Big &b) {
        Big r;
        if (!cuboid::add(a, b, r)) ok = false;
        return r;
    }
    Big pow(const Big &a, int e) {
        Big r = Big::from_u64(1);
        for (int i = 0; i < e; ++i) r = mul(r, a);
        return r;
    }
    Big scal(int64_t k, const Big &a) {
        Big kk = Big::from_u64((uint64_t)(k < 0 ? -k : k));
        kk.neg = k < 0;
        return mul(kk, a);
    }
};

std::string to_decimal(Big v) {
    if (v.is_zero()) return "0";
    const bool negative = v.neg;
    std::string digits;
    while (!v.is_zero()) {
        // divide magnitude by 10^18
        const uint64_t base = 1000000000000000000ull;
        u128 rem = 0;
        for (int i = kLimbs - 1; i >= 0; --i) {
            u128 cur = (rem << 64) | v.l[i];
            v.l[i] = (uint64_t)(cur / base);
            rem = cur % base;
        }
        char buf[32];
        uint64_t r = (uint64_t)rem;
        for (int k = 0; k < 18; ++k) {
            buf[k] = (char)('0' + r % 10);
            r /= 10;
        }
        digits.append(buf, 18);
    }
    while (digits.size() > 1 && digits.back() == '0') digits.pop_back();
    if (negative) digits.push_back('-');
    std::reverse(digits.begin(), digits.end());
    return digits;
}

}  // namespace

// Q_pq(t) exactly, from the factored coefficients of eq. (1.1).
static bool q_exact(uint32_t p, uint32_t q, uint64_t t_lo, uint64_t t_hi, Big &out) {
    Ctx c;
    const Big P = Big::from_u64((uint64_t)p * p), Q = Big::from_u64((uint64_t)q * q);
    const Big t = Big::from_i128(false, (u128)t_hi << 64 | t_lo);
    const Big s = c.mul(t, t);
    const Big P2 = c.pow(P, 2), P3 = c.pow(P, 3), P4 = c.pow(P, 4), P5 = c.pow(P, 5);
    const Big Q2 = c.pow(Q, 2), Q3 = c.pow(Q, 3), Q4 = c.pow(Q, 4), Q5 = c.pow(Q, 5);
    // s^4: (2Q + P)(3Q - 2P)
    const Big c8 = c.mul(c.add(c.scal(2, Q), P), c.add(c.scal(3, Q), c.scal(-2, P)));
    // s^3: Q^4 + 10 P Q^3 + 4 P^2 Q^2 - 14 P^3 Q + P^4
    Big c6 = c.add(Q4, c.scal(10, c.mul(P, Q3)));
    c6 = c.add(c6, c.scal(4, c.mul(P2, Q2)));
    c6 = c.add(c6, c.scal(-14, c.mul(P3, Q)));
    c6 = c.add(c6, P4);
    // s^2: -P Q (Q^4 - 14 P Q^3 + 4 P^2 Q^2 + 10 P^3 Q + P^4)
    Big in4 = c.add(Q4, c.scal(-14, c.mul(P, Q3)));
    in4 = c.add(in4, c.scal(4, c.mul(P2, Q2)));
    in4 = c.add(in4, c.scal(10, c.mul(P3, Q)));
    in4 = c.add(in4, P4);
    const Big c4 = negate(c.mul(c.mul(P, Q), in4));
    // s^1: -P^3 Q^3 (Q + 2P)(3P - 2Q)
    const Big c2 = negate(c.mul(c.mul(P3, Q3),
                                c.mul(c.add(Q, c.scal(2, P)), c.add(c.scal(3, P), c.scal(-2, Q)))));
    // s^0: -P^5 Q^5
    const Big c0 = negate(c.mul(P5, Q5));
    Big v = c.add(s, c8);
    v = c.add(c.mul(v, s), c6);
    v = c.add(c.mul(v, s), c4);
    v = c.add(c.mul(v, s), c2);
    v = c.add(c.mul(v, s), c0);
    out = v;
    return c.ok;
}

uint32_t theorem_flags(uint32_t p, uint32_t q, uint64_t t_lo, uint64_t t_hi) {
    const u128 p2 = (u128)p * p, pq = (u128)p * q, q2 = (u128)q * q;
    const u128 tt = (u128)t_hi << 64 | t_lo;
    uint32_t f = 0;
    if (tt > p2) f |= 1;
    if (tt > pq) f |= 2;
    if (tt > q2) f |= 4;
    // (p^2 + t)(pq + t) > 2 t^2: both sides below 2^260 for t < 2^128, as Big
    Ctx c;
    const Big T = Big::from_i128(false, tt);
    const Big lhs = c.mul(c.add(Big::from_i128(false, p2), T), c.add(Big::from_i128(false, pq), T));
    const Big rhs = c.scal(2, c.mul(T, T));
    if (cmp_mag(lhs, rhs) > 0) f |= 8;
    return f;
}

bool exact_is_root(uint32_t p, uint32_t q, uint64_t t_lo, uint64_t t_hi, bool *ok) {
    Big v;
    *ok = t_hi < 64 && q_exact(p, q, t_lo, t_hi, v);
    return *ok && v.is_zero();
}

bool exact_value_decimal(uint32_t p, uint32_t q, uint64_t t_lo, uint64_t t_hi, std::string *out) {
    Big v;
    if (t_hi >= 64 || !q_exact(p, q, t_lo, t_hi, v)) return false;
    *out = to_decimal(v);
    return true;
}

}  // namespace cuboid
