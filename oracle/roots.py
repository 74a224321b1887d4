"""ORACLE — test infrastructure only (never imported by the product library).

Exact search for the positive integer roots t of Q_pq(t) = 0 (eq. 1.1 of
Gallyamov et al., arXiv:1601.00636), the question Theorem 1.1 turns a perfect
cuboid into.

Method (deliberately unlike the divisor enumeration the GPU path uses): real
root isolation of P(s) = Q_pq(sqrt(s)) with Python integers.  The real roots of
a polynomial's derivative split the line into pieces on which the polynomial
is monotone; each piece holds at most one root, located by integer bisection on
the exact sign.  Recursing down the derivatives gives, for every real root, an
integer interval [k, k+1] containing it, so every integer root is among a short
list of candidates that are then tested exactly.  Q is even in t, so the
positive integer roots t are the integer square roots of the positive
integer roots s that are perfect squares.
"""
from math import isqrt

from .poly import q_coeffs, theorem_1_1_flags


def _trim(a):
    a = list(a)
    while a and a[-1] == 0:
        a.pop()
    return a


def _eval(a, x):
    v = 0
    for c in reversed(a):
        v = v * x + c
    return v


def _deriv(a):
    return [i * a[i] for i in range(1, len(a))]


def _sign(v):
    return (v > 0) - (v < 0)


def _floor_candidates(a):
    """A set of integers containing floor(x) for every real root x of a
    (coefficients ascending).  Supersets are fine: callers test exactly."""
    a = _trim(a)
    n = len(a) - 1
    if n <= 0:
        return set()
    if n == 1:
        return {(-a[0]) // a[1]}
    crit = _floor_candidates(_deriv(a))
    # Cauchy bound: every root has |x| <= 1 + max |a_i / a_n|
    bound = 2 + max(abs(c) for c in a[:-1]) // abs(a[-1])
    pts = {-bound, bound}
    for k in crit:
        for x in (k, k + 1):
            if -bound <= x <= bound:
                pts.add(x)
    pts = sorted(pts)
    out = set()
    for lo, hi in zip(pts[:-1], pts[1:]):
        if hi - lo == 1:
            # may hold a critical point: keep both ends as candidates
            out.update((lo, hi))
            continue
        flo, fhi = _eval(a, lo), _eval(a, hi)
        if flo == 0:
            out.add(lo)
        if fhi == 0:
            out.add(hi)
        if _sign(flo) * _sign(fhi) < 0:
            # monotone with a sign change: exactly one root strictly inside
            while hi - lo > 1:
                mid = (lo + hi) // 2
                fm = _eval(a, mid)
                if fm == 0:
                    out.add(mid)
                    break
                if _sign(fm) == _sign(flo):
                    lo, flo = mid, fm
                else:
                    hi = mid
            else:
                out.update((lo, hi))
    return out


def integer_roots(a):
    """All integer roots of the nonzero integer polynomial a (ascending)."""
    a = _trim(a)
    if not a:
        raise ValueError("zero polynomial")
    return sorted(k for k in _floor_candidates(a) if _eval(a, k) == 0)


def positive_t_roots(p, q):
    """Sorted positive integers t with Q_pq(t) = 0 exactly."""
    out = []
    for s in integer_roots(q_coeffs(p, q)):
        if s > 0:
            t = isqrt(s)
            if t * t == s:
                out.append(t)
    return out


def root_check(pairs):
    """For each (p, q): every positive integer root t with its Theorem 1.1 flag
    bits, as (p, q, t, flags) tuples in input order, roots ascending."""
    res = []
    for p, q in pairs:
        for t in positive_t_roots(p, q):
            res.append((int(p), int(q), int(t), theorem_1_1_flags(p, q, t)))
    return res
