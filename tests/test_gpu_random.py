"""Randomized differential checks against the oracle: seeded random prime
lists (ascending or shuffled, 1 to 39 primes below 1000) and rectangles of
several shapes (small squares, 64-row strips up to 20000 columns, rows and
columns at 2^24, 2^31 and 2^32 - 1, near-diagonal squares), through the plain
call, the batched call and region slices with random bands."""
import numpy as np
import pytest

import oracle
from paper_1601_00636_amd import binding as cb

pytestmark = pytest.mark.gpu

M = 2**32 - 1
SMALL = [r for r in range(3, 1000) if all(r % d for d in range(2, int(r ** 0.5) + 1))]


@pytest.fixture(scope="module")
def ctx():
    h = cb.cuboid_create(0)
    yield h
    assert cb.cuboid_destroy(h) == cb.OK


def _primes(rng):
    ps = sorted(int(x) for x in rng.choice(SMALL, size=int(rng.integers(1, 40)), replace=False))
    if rng.random() < 0.3:
        rng.shuffle(ps)
    return ps


def _rect(rng):
    kind = rng.integers(0, 5)
    if kind == 0:
        p0, q0 = int(rng.integers(1, 5000)), int(rng.integers(1, 5000))
        return (p0, p0 + int(rng.integers(0, 300)), q0, q0 + int(rng.integers(0, 300)))
    if kind == 1:
        p0, q0 = int(rng.integers(1, 10**6)), int(rng.integers(1, 10**6))
        return (p0, p0 + int(rng.integers(0, 64)), q0, q0 + int(rng.integers(0, 20000)))
    if kind == 2:
        p0 = int(rng.choice([2**24 - 100, 2**31 - 100, M - 300])) + int(rng.integers(0, 90))
        q0 = int(rng.integers(1, 10**6))
        return (p0, min(M, p0 + int(rng.integers(0, 100))), q0, q0 + int(rng.integers(0, 1000)))
    if kind == 3:
        q0 = int(rng.choice([2**24 - 50, 2**31 - 50, M - 2000]))
        p0 = int(rng.integers(1, 10**5))
        return (p0, p0 + int(rng.integers(0, 200)), q0, min(M, q0 + int(rng.integers(0, 1500))))
    p0 = int(rng.integers(1, 3000))
    return (p0, p0 + int(rng.integers(0, 2000)), p0, p0 + int(rng.integers(0, 2000)))


def _same(g, o):
    assert g["n_pairs"] == o["n_pairs"]
    assert [int(x) for x in g["counts"]] == [int(x) for x in o["counts"]]
    assert [int(x) for x in g["survivors"]] == [int(x) for x in o["survivors"]]


@pytest.mark.parametrize("seed", [101, 202])
def test_random_plain_and_batched(ctx, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    for n in range(400):
        primes = _primes(rng)
        rect = _rect(rng)
        _same(cb.cuboid_sieve_range(ctx, *rect, primes, cap=1 << 21),
              oracle.sieve(*rect, primes, cap=1 << 21))
        if n % 10 == 0:
            rects = [_rect(rng) for _ in range(int(rng.integers(2, 20)))]
            st, out = cb.cuboid_sieve_batch(ctx, rects, primes, caps=1 << 21)
            assert st == cb.OK
            for r, x in zip(rects, out):
                _same(x, oracle.sieve(*r, primes, cap=1 << 21))


@pytest.mark.parametrize("seed", [303])
def test_random_region_slices(ctx, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    for _ in range(40):
        primes = _primes(rng)
        rp = sorted(set([r for r in primes if r >= 11] + [11, 13, 17, 19, 23, 29, 31, 37]))
        if rng.random() < 0.5:
            rng.shuffle(rp)
        p0 = int(rng.integers(1, 5000))
        p1 = p0 + int(rng.integers(0, 60))
        band = int(rng.integers(1, 80))
        got = cb.cuboid_sieve_region(ctx, p0, p1, rp, band_rows=band, cap=1 << 22)
        ref = oracle.sieve_region(p0, p1, rp)
        by_prime = dict(zip(sorted(rp), [int(c) for c in ref["counts"]]))
        assert got["n_pairs"] == ref["n_pairs"]
        assert [int(c) for c in got["counts"]] == [by_prime[r] for r in rp]
        assert got["survivors"] == ref["survivors"]
