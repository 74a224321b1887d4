"""Served form: continuous batching keeps every result bit-exact.

Each request's counts, pair count and sorted survivors from the server equal
those of the plain call on the same rectangle alone (and the oracle's on the
small ones), whatever the mix, slot count, launch size or memory budget.
"""
import time

import numpy as np
import pytest

import oracle
from paper_1601_00636_amd import binding as cb
from paper_1601_00636_amd import workloads as wl

pytestmark = pytest.mark.gpu

PRIMES = wl.PRIMES_BATCHED


@pytest.fixture(scope="module")
def ctx():
    h = cb.cuboid_create(0)
    yield h
    assert cb.cuboid_destroy(h) == cb.OK


def _same(a, b):
    assert a["n_pairs"] == b["n_pairs"]
    assert [int(x) for x in a["counts"]] == [int(x) for x in b["counts"]]
    assert [int(x) for x in a["survivors"]] == [int(x) for x in b["survivors"]]


def _mix(seed, n, big=()):
    rng = np.random.Generator(np.random.PCG64(seed))
    rects = []
    for _ in range(n):
        h = int(np.exp(rng.uniform(0, np.log(3000))))
        w = int(np.exp(rng.uniform(0, np.log(3000))))
        p0 = int(rng.integers(1, 10**6))
        q0 = int(rng.integers(1, 10**6))
        rects.append((p0, p0 + h - 1, q0, q0 + w - 1))
    return list(big) + rects


def test_server_matches_plain_and_oracle(ctx):
    rects = _mix(1, 150, big=[(1, 20000, 1, 20000)])
    rects += [(1, 200, 1, 200), (5, 5, 5, 5), (1, 1, 1, 3)]
    srv = cb.cuboid_server_start(ctx, PRIMES, streams=2, max_launch_units=1 << 14)
    try:
        tickets = [cb.cuboid_server_submit(srv, r) for r in rects]
        got = [cb.cuboid_server_poll(srv, t, len(PRIMES), cap=4096) for t in tickets]
        stats = cb.cuboid_server_stats_get(srv)
    finally:
        cb.cuboid_server_stop(srv)
    assert stats["completed"] == len(rects) and stats["launches"] > 2
    for rect, g in zip(rects, got):
        assert g["status"] == cb.OK
        _same(g, cb.cuboid_sieve_range(ctx, *rect, PRIMES, cap=4096))
    for rect, g in list(zip(rects, got))[-4:]:
        _same(g, oracle.sieve(*rect, PRIMES))


def test_small_requests_overtake_a_large_one(ctx):
    big = (1, 60000, 1, 60000)        # ~880k units: many launches of 2^14 units
    small = _mix(2, 60)
    srv = cb.cuboid_server_start(ctx, PRIMES, streams=2, max_launch_units=1 << 14)
    try:
        tb = cb.cuboid_server_submit(srv, big)
        time.sleep(0.002)
        ts = [cb.cuboid_server_submit(srv, r) for r in small]
        gs = [cb.cuboid_server_poll(srv, t, len(PRIMES)) for t in ts]
        gb = cb.cuboid_server_poll(srv, tb, len(PRIMES))
        stats = cb.cuboid_server_stats_get(srv)
    finally:
        cb.cuboid_server_stop(srv)
    # admitted while the big one was on the GPU, and finished before it
    assert stats["max_admitted"] > 1
    assert max(g["done_ns"] for g in gs) < gb["done_ns"]
    assert min(g["admit_ns"] for g in gs) < gb["done_ns"]
    _same(gb, cb.cuboid_sieve_range(ctx, *big, PRIMES))
    for r, g in zip(small, gs):
        _same(g, cb.cuboid_sieve_range(ctx, *r, PRIMES))


def test_admission_under_small_budget_and_few_slots(ctx):
    rects = _mix(3, 40, big=[(1000, 9000, 1, 5000)])
    # 64 KiB of row-order memory: requests wait for each other; the first one
    # (8001 rows, 32 KiB) fits, any larger one would run in row order
    srv = cb.cuboid_server_start(ctx, PRIMES, streams=3, max_slots=3, max_launch_units=1 << 12,
                                 hbm_budget_bytes=1 << 16)
    try:
        ts = [cb.cuboid_server_submit(srv, r) for r in rects]
        gs = [cb.cuboid_server_poll(srv, t, len(PRIMES)) for t in ts]
        stats = cb.cuboid_server_stats_get(srv)
    finally:
        cb.cuboid_server_stop(srv)
    assert stats["max_admitted"] <= 3
    for r, g in zip(rects, gs):
        _same(g, cb.cuboid_sieve_range(ctx, *r, PRIMES))


def test_request_larger_than_arena_runs_in_row_order(ctx):
    rect = (1, 40000, 7, 900)          # 160 KB of row order > 64 KiB arena
    srv = cb.cuboid_server_start(ctx, PRIMES, hbm_budget_bytes=1 << 16)
    try:
        g = cb.cuboid_server_poll(srv, cb.cuboid_server_submit(srv, rect), len(PRIMES))
    finally:
        cb.cuboid_server_stop(srv)
    _same(g, cb.cuboid_sieve_range(ctx, *rect, PRIMES))


def test_capacity_retry_and_errors(ctx):
    srv = cb.cuboid_server_start(ctx, wl.PRIMES_C1)
    try:
        t = cb.cuboid_server_submit(srv, (1, 200, 1, 200))
        with pytest.raises(cb.CuboidError) as e:
            cb.cuboid_server_poll(srv, t, len(wl.PRIMES_C1), cap=3)
        assert e.value.status == cb.E_CAPACITY and e.value.needed == 26
        g = cb.cuboid_server_poll(srv, t, len(wl.PRIMES_C1), cap=64)
        _same(g, oracle.sieve(1, 200, 1, 200, wl.PRIMES_C1))
        with pytest.raises(cb.CuboidError) as e:
            cb.cuboid_server_poll(srv, t, len(wl.PRIMES_C1))     # handed out already
        assert e.value.status == cb.E_ARG
        with pytest.raises(cb.CuboidError) as e:
            cb.cuboid_server_submit(srv, (5, 4, 1, 1))
        assert e.value.status == cb.E_RANGE
        assert cb.cuboid_destroy(ctx) == cb.E_BUSY            # a server is running
        t2 = cb.cuboid_server_submit(srv, (3, 300, 7, 500))
        assert cb.cuboid_server_poll(srv, t2, len(wl.PRIMES_C1), wait=True) is not None
    finally:
        cb.cuboid_server_stop(srv)


def test_submit_many(ctx):
    # a batch of requests queued in one call gives the same results as one
    # call per request; an invalid rectangle queues none of its batch
    rects = _mix(7, 120) + [(1, 200, 1, 200), (9, 9, 1, 1)]
    srv = cb.cuboid_server_start(ctx, PRIMES, streams=2, max_launch_units=1 << 14)
    try:
        before = cb.cuboid_server_stats_get(srv)["submitted"]
        with pytest.raises(cb.CuboidError) as e:
            cb.cuboid_server_submit_many(srv, [(1, 5, 1, 5), (6, 5, 1, 1), (1, 1, 1, 2)])
        assert e.value.status == cb.E_RANGE and e.value.needed == 1
        assert cb.cuboid_server_stats_get(srv)["submitted"] == before
        tickets = cb.cuboid_server_submit_many(srv, rects)
        assert len(set(int(t) for t in tickets)) == len(rects)
        got = [cb.cuboid_server_poll(srv, int(t), len(PRIMES), cap=4096) for t in tickets]
        stats = cb.cuboid_server_stats_get(srv)
    finally:
        cb.cuboid_server_stop(srv)
    assert stats["completed"] == len(rects) and stats["max_admitted"] > 1
    for rect, g in zip(rects, got):
        assert g["status"] == cb.OK
        _same(g, cb.cuboid_sieve_range(ctx, *rect, PRIMES, cap=4096))
    _same(got[-2], oracle.sieve(1, 200, 1, 200, PRIMES))


def test_poisson_replay_small(ctx):
    stream = wl.served_stream(duration=0.3, max_requests=600, area_hi=1e7)
    srv = cb.cuboid_server_start(ctx, PRIMES)
    try:
        t0 = time.perf_counter()
        tickets = []
        for at, rect in stream:
            while time.perf_counter() - t0 < at:
                pass
            tickets.append(cb.cuboid_server_submit(srv, rect))
        res = [cb.cuboid_server_poll(srv, t, len(PRIMES), cap=4096) for t in tickets]
    finally:
        cb.cuboid_server_stop(srv)
    lat = np.array([r["latency_ns"] for r in res]) / 1e6
    print("served %d requests: p50 %.3f ms p99 %.3f ms" % (len(res), np.percentile(lat, 50),
                                                           np.percentile(lat, 99)))
    for (_, rect), r in list(zip(stream, res))[::25]:
        _same(r, cb.cuboid_sieve_range(ctx, *rect, PRIMES, cap=4096))


def test_survivor_pool_overflow_is_swept_again(ctx):
    # with the prime 11 alone about a third of the pairs survive: requests of
    # ~2e5 survivors each overflow the 2^16-entry pool of a launch, which is
    # then swept again with a larger pool; every list is complete, counts
    # are counted once
    primes = [11]
    rects = [(1, 1000, 1, 1000), (5000, 5600, 20000, 20900), (1, 40, 1, 40),
             (70000, 70700, 3, 800)]
    srv = cb.cuboid_server_start(ctx, primes, streams=2, max_launch_units=1 << 9)
    try:
        ts = [cb.cuboid_server_submit(srv, r) for r in rects]
        got = [cb.cuboid_server_poll(srv, t, 1, cap=1 << 20) for t in ts]
        stats = cb.cuboid_server_stats_get(srv)
    finally:
        cb.cuboid_server_stop(srv)
    assert stats["resweeps"] > 0
    for rect, g in zip(rects, got):
        assert g["status"] == cb.OK
        ref = oracle.sieve(*rect, primes, cap=1 << 20)
        _same(g, ref)
    assert max(g["n_survivors"] for g in got) > 1 << 16


def test_rows_beyond_the_resident_table(ctx):
    # p above 2^24 up to 2^32 - 1: each request's rows are factored into the
    # arena at its first launch; against the oracle
    primes = wl.PRIMES_C1
    rects = [(2**31, 2**31 + 300, 5, 900), (2**32 - 200, 2**32 - 1, 1, 500),
             (16777200, 16777300, 1, 700), (3000000019, 3000000019, 2999999000, 3000001000),
             (1, 200, 1, 200)]
    srv = cb.cuboid_server_start(ctx, primes, streams=2, max_launch_units=1 << 8)
    try:
        ts = [cb.cuboid_server_submit(srv, r) for r in rects]
        got = [cb.cuboid_server_poll(srv, t, len(primes), cap=1 << 16) for t in ts]
    finally:
        cb.cuboid_server_stop(srv)
    for rect, g in zip(rects, got):
        assert g["status"] == cb.OK
        _same(g, oracle.sieve(*rect, primes, cap=1 << 16))


def test_row_table_larger_than_the_arena(ctx):
    # a request whose own row table cannot fit the arena finishes with E_LIMIT
    srv = cb.cuboid_server_start(ctx, wl.PRIMES_C1, hbm_budget_bytes=1 << 16)
    try:
        t = cb.cuboid_server_submit(srv, (2**31, 2**31 + 10000, 1, 10))
        with pytest.raises(cb.CuboidError) as e:
            cb.cuboid_server_poll(srv, t, len(wl.PRIMES_C1))
        assert e.value.status == cb.E_LIMIT
        t2 = cb.cuboid_server_submit(srv, (2**31, 2**31 + 100, 1, 300))
        g = cb.cuboid_server_poll(srv, t2, len(wl.PRIMES_C1))
    finally:
        cb.cuboid_server_stop(srv)
    _same(g, oracle.sieve(2**31, 2**31 + 100, 1, 300, wl.PRIMES_C1))
