"""Deep prime lists: tables up to the paper's format limit (eq. 2.7, r < 9697)
and beyond, up to the largest prime below 2^16, and sieves whose lists hold
more than a thousand primes, against the table-free oracle (Definition 1.1
evaluated entry by entry).
"""
import numpy as np
import pytest

import oracle
from paper_1601_00636_amd import binding as cb
from paper_1601_00636_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    h = cb.cuboid_create(0)
    yield h
    assert cb.cuboid_destroy(h) == cb.OK


def _bits(raw, r):
    b = np.unpackbits(np.frombuffer(raw, dtype=np.uint8), bitorder="little")[: r * r]
    return b.reshape(r, r)


@pytest.mark.parametrize("r", [1009, 4099, 9689, 9697])
def test_large_tables_sampled_and_density(ctx, r):
    u = _bits(bytes(cb.cuboid_table_bytes(ctx, r)), r)
    rng = np.random.Generator(np.random.PCG64(r))
    for a, b in rng.integers(0, r, size=(150, 2)):
        assert u[a, b] == oracle.u_entry(int(a), int(b), r), (a, b)
    if r != 9689:
        # density: each ratio class a/b = x of F_r* fills r - 1 entries, so the
        # popcount is (r - 1) times the classes with u(x, 1) = 1
        classes = sum(oracle.u_entry(x, 1, r) for x in range(1, r))
        assert int(u.sum()) == (r - 1) * classes


def test_sieve_with_the_primes_up_to_9697(ctx):
    primes = wl.primes_upto(9697, 11)
    assert len(primes) == 1193 and primes[-1] == 9697
    for rect in ((1, 150, 1, 150), (90000, 90060, 123456, 123700)):
        ref = oracle.sieve(*rect, primes, direct=True)
        got = cb.cuboid_sieve_range(ctx, *rect, primes)
        assert got["n_pairs"] == ref["n_pairs"]
        assert [int(c) for c in got["counts"]] == [int(c) for c in ref["counts"]]
        assert [int(x) for x in got["survivors"]] == [int(x) for x in ref["survivors"]]


def test_sieve_with_the_largest_primes_below_2_16(ctx):
    primes = [11, 13, 17, 65521, 65519, 65497, 40009]
    rect = (1, 60, 1, 70)
    ref = oracle.sieve(*rect, primes, direct=True)
    got = cb.cuboid_sieve_range(ctx, *rect, primes, cap=1 << 12)
    assert got["n_pairs"] == ref["n_pairs"]
    assert [int(c) for c in got["counts"]] == [int(c) for c in ref["counts"]]
    assert [int(x) for x in got["survivors"]] == [int(x) for x in ref["survivors"]]
    assert sum(int(c) for c in got["counts"][3:]) > 0     # the large primes do reject
