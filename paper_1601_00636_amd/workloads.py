"""Seeded synthetic inputs for the cuboid sieve: rectangles of (p, q) pairs,
prime lists, batches of rectangles and Poisson request streams.

This module draws inputs only; it holds none of the sieve's arithmetic and is
shared by the tests, the benchmark and the serving driver.  The paper
(arXiv:1601.00636) scans region (1.2) with no external dataset; everything here
is generated from numpy PCG64 streams with a recorded seed.
"""
import numpy as np

SEED = 20160401


def primes_upto(hi, lo=2):
    """Primes lo <= r <= hi, by trial division (input preparation only)."""
    out = []
    for r in range(max(2, lo), hi + 1):
        d, ok = 2, True
        while d * d <= r:
            if r % d == 0:
                ok = False
                break
            d += 1
        if ok:
            out.append(r)
    return out


PRIMES_C1 = primes_upto(31, 3)        # the 10 smallest odd primes
PRIMES_C2 = primes_upto(97, 3)        # 24 primes, 3 <= r < 100
PRIMES_C3 = primes_upto(997, 3)       # 167 primes, 3 <= r < 1000
PRIMES_BATCHED = primes_upto(499, 3)  # 94 primes, 3 <= r < 500
PRIMES_PAPER = primes_upto(541, 11)   # the paper's 96 primes 11..541 (section 2)

SQUARES = {
    # name: (side, primes) for the square [1, side]^2
    "c1": (200, PRIMES_C1),
    "c2": (10**4, PRIMES_C2),
    "c3": (10**5, PRIMES_C3),
}


def square(name):
    """(p0, p1, q0, q1, primes) for one of the square workloads."""
    n, primes = SQUARES[name]
    return 1, n, 1, n, list(primes)


def batched_requests(n=4096, seed=SEED, side_lo=32, side_hi=3 * 10**4, origin_hi=10**6):
    """n rectangles (p0, p1, q0, q1), inclusive bounds.

    Side lengths floor(exp(U(ln side_lo, ln side_hi))) drawn independently for
    the p and q sides; origins uniform on 1..origin_hi.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = np.log(side_lo), np.log(side_hi)
    hp = np.floor(np.exp(rng.uniform(lo, hi, n))).astype(np.int64)
    hq = np.floor(np.exp(rng.uniform(lo, hi, n))).astype(np.int64)
    p0 = rng.integers(1, origin_hi + 1, n)
    q0 = rng.integers(1, origin_hi + 1, n)
    return [(int(a), int(a + h - 1), int(b), int(b + w - 1))
            for a, h, b, w in zip(p0, hp, q0, hq)]


def served_stream(seed=SEED + 1, rate=2000.0, duration=10.0, max_requests=20000,
                  area_lo=1e3, area_hi=1e9, aspect=16.0, origin_hi=10**6):
    """A Poisson request stream: list of (arrival_seconds, (p0, p1, q0, q1)).

    Exponential inter-arrival times with mean 1/rate; areas log-uniform in
    [area_lo, area_hi]; aspect ratio (rows / columns) log-uniform in
    [1/aspect, aspect]; sides rounded, at least 1; origins uniform on
    1..origin_hi.  Stops at `duration` seconds or `max_requests` requests.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    t = 0.0
    while len(out) < max_requests:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        area = np.exp(rng.uniform(np.log(area_lo), np.log(area_hi)))
        asp = np.exp(rng.uniform(-np.log(aspect), np.log(aspect)))
        h = max(1, int(round(np.sqrt(area * asp))))
        w = max(1, int(round(np.sqrt(area / asp))))
        p0 = int(rng.integers(1, origin_hi + 1))
        q0 = int(rng.integers(1, origin_hi + 1))
        out.append((t, (p0, p0 + h - 1, q0, q0 + w - 1)))
    return out


def random_rectangles(n, seed, max_coord=2000, max_side=300):
    """Small random rectangles for property tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n):
        h = int(rng.integers(1, max_side + 1))
        w = int(rng.integers(1, max_side + 1))
        p0 = int(rng.integers(1, max_coord + 1))
        q0 = int(rng.integers(1, max_coord + 1))
        out.append((p0, p0 + h - 1, q0, q0 + w - 1))
    return out
