"""The allocation-free batched sieve (cuboid_sieve_batch_dev_noalloc) against
the regular one (cuboid_sieve_batch_dev) through the C interface: counts,
pair counts and sorted survivor lists equal, on two calls in a row (the
second smaller, so that anything the first left in the shared scratch array
would show), plus its refusals."""
import numpy as np
import pytest

from paper_1601_00636_amd import binding as cb
from paper_1601_00636_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    h = cb.cuboid_create(0)
    yield h
    assert cb.cuboid_destroy(h) == cb.OK


def _same(dev_a, dev_b):
    ca, pa, sa = dev_a.read()
    cb_, pb, sb = dev_b.read()
    assert dev_a.n_survivors == dev_b.n_survivors
    assert np.array_equal(ca, cb_)
    assert np.array_equal(pa, pb)
    assert np.array_equal(sa["idx"], sb["idx"]) and np.array_equal(sa["req"], sb["req"])
    return ca, pa, sa


def _run_both(ctx, rects, primes, surv_cap):
    ref = cb.DeviceBatch(ctx, len(rects), len(primes), surv_cap=surv_cap)
    got = cb.DeviceBatch(ctx, len(rects), len(primes), surv_cap=surv_cap)
    try:
        st_ref = cb.cuboid_sieve_batch_dev(ctx, rects, primes, ref)
        st_got = cb.cuboid_sieve_batch_dev_noalloc(ctx, rects, primes, got)
        assert st_got == st_ref
        return st_got, _same(got, ref)
    finally:
        ref.free()
        got.free()


def test_two_calls_in_a_row_equal_the_regular_path(ctx):
    primes = wl.PRIMES_C1          # survivors in most rectangles
    big = wl.random_rectangles(300, seed=901, max_coord=20000, max_side=600) + [(1, 200, 1, 200)]
    small = wl.random_rectangles(37, seed=902, max_coord=3000, max_side=90)
    # the tables and the row table come from an earlier regular call
    cb.cuboid_sieve_range(ctx, 20600, 20600, 1, 1, primes)
    st, (c1, p1, s1) = _run_both(ctx, big, primes, 1 << 16)
    assert st == cb.OK and len(s1) > 26 and int(p1.sum()) > 0
    st, (c2, p2, s2) = _run_both(ctx, small, primes, 1 << 16)
    assert st == cb.OK and len(p2) == 37
    # and a survivor capacity below the count: the first ones, E_CAPACITY
    st, _ = _run_both(ctx, big, primes, 5)
    assert st == cb.E_CAPACITY


def test_batched_workload_with_its_primes(ctx):
    # the benchmark's 4096 rectangles (rows regrouped until the array's
    # row-order part is full), then a smaller batch
    primes = wl.PRIMES_BATCHED
    reqs = wl.batched_requests(4096)
    cb.cuboid_sieve_range(ctx, 1030000, 1030000, 1, 1, primes)
    st, (c, p, s) = _run_both(ctx, reqs, primes, 1 << 12)
    assert st == cb.OK and int(p.sum()) == 46463395437
    st, _ = _run_both(ctx, reqs[:100], primes, 1 << 12)
    assert st == cb.OK


def test_refusals(ctx):
    fresh = cb.cuboid_create(0)
    try:
        primes = [11, 13, 17]
        dev = cb.DeviceBatch(fresh, 1, 3, surv_cap=16)
        try:
            # tables not built on this context yet: nothing is built here
            with pytest.raises(cb.CuboidError) as e:
                cb.cuboid_sieve_batch_dev_noalloc(fresh, [(1, 50, 1, 50)], primes, dev)
            assert e.value.status == cb.E_NOT_LOADED
            cb.cuboid_sieve_range(fresh, 1, 50, 1, 50, primes)
            # rows past the resident table (checked on the host)
            assert cb.cuboid_sieve_batch_dev_noalloc(fresh, [(1, 2**25, 1, 50)], primes,
                                                     dev) == cb.E_LIMIT
            with pytest.raises(cb.CuboidError) as e:
                cb.cuboid_sieve_batch_dev_noalloc(fresh, [(0, 5, 1, 50)], primes, dev)
            assert e.value.status == cb.E_RANGE
            # and a valid call still works after the refusals
            assert cb.cuboid_sieve_batch_dev_noalloc(fresh, [(1, 50, 1, 50)], primes,
                                                     dev) in (cb.OK, cb.E_CAPACITY)
        finally:
            dev.free()
        # more requests than the array's descriptors alone hold (96 bytes each
        # against 64 MiB): refused on the host before any device work
        n = 1000000
        big = cb.DeviceBatch(fresh, n, 3, surv_cap=0)
        try:
            reqs = np.tile(np.array([[1, 50, 1, 50]], dtype=np.uint32), (n, 1))
            assert cb.cuboid_sieve_batch_dev_noalloc(fresh, reqs, primes, big) == cb.E_LIMIT
        finally:
            big.free()
    finally:
        assert cb.cuboid_destroy(fresh) == cb.OK
