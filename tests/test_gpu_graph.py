"""Captured-graph launches against call-by-call launches.

Plain and batched calls over resident rows replay a captured HIP graph by
default.  Each replay must equal, element by element, what the same call
gives with graphs off (a second context), also when other GPU work and
synchronizations run between replays, when the cache evicts graphs, and with
event nodes timing the sweep.  The call-by-call path is checked against the
oracle on its own.
"""
import numpy as np
import pytest

import oracle
from paper_1601_00636_amd import binding as cb
from paper_1601_00636_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pair():
    g = cb.cuboid_create(0)
    e = cb.cuboid_create(0)
    cb.cuboid_enable_graphs(e, False)
    yield g, e
    assert cb.cuboid_destroy(g) == cb.OK
    assert cb.cuboid_destroy(e) == cb.OK


def _same_batch(a, b):
    assert list(a.n_pairs) == list(b.n_pairs)
    assert np.array_equal(a.counts, b.counts)
    assert list(a.n_survivors) == list(b.n_survivors)
    assert list(a.status) == list(b.status)
    for i in range(len(a.n_pairs)):
        sa, sb = a[i]["survivors"], b[i]["survivors"]
        assert (sa is None) == (sb is None)
        if sa is not None:
            assert [int(x) for x in sa] == [int(x) for x in sb]


def _cmp(res, ref):
    assert res["n_pairs"] == ref["n_pairs"]
    assert [int(x) for x in res["counts"]] == [int(x) for x in ref["counts"]]
    assert [int(x) for x in res["survivors"]] == [int(x) for x in ref["survivors"]]


def _batch(seed, n):
    rects = wl.random_rectangles(n, seed=seed, max_coord=300000, max_side=3000)
    return rects + [(1, 200, 1, 200), (5, 5, 5, 5)]


def test_replays_match_call_by_call(pair):
    g, e = pair
    primes = wl.PRIMES_C2
    # buffers grown to what the interleaved calls need, so that only the
    # first batch captures (a grown buffer means a new capture)
    cb.cuboid_sieve_range(g, 3, 900, 7, 1100, primes)
    cb.cuboid_enable_timing(g, True)
    kinds = []
    try:
        for seed in range(5):
            rects = _batch(100 + seed, 198)
            st_g, out_g = cb.cuboid_sieve_batch(g, rects, primes, caps=64)
            kinds.append(cb.cuboid_last_timing(g)["graph"])
            st_e, out_e = cb.cuboid_sieve_batch(e, rects, primes, caps=64)
            assert st_g == st_e == cb.OK
            _same_batch(out_g, out_e)
            # other work on the same context and device between replays
            one = cb.cuboid_sieve_range(g, 3, 900, 7, 1100, primes)
            _cmp(one, cb.cuboid_sieve_range(e, 3, 900, 7, 1100, primes))
            qm = cb.cuboid_q_mod_prime(g, [seed + 1] * 4, [2, 3, 4, 5], [0, 1, 2, 3], [11, 13, 17, 19])
            assert len(qm) == 4
    finally:
        cb.cuboid_enable_timing(g, False)
    # captured once, then replayed for every later batch of the same shape
    assert kinds[0] == 2 and kinds[1:] == [1, 1, 1, 1]


def test_sweep_timing_inside_the_graph(pair):
    g, _ = pair
    primes = wl.PRIMES_C3
    cb.cuboid_enable_timing(g, True)
    try:
        for _ in range(3):
            res = cb.cuboid_sieve_range(g, 1, 20000, 1, 20000, primes)
            t = cb.cuboid_last_timing(g)
            assert t["graph"] in (1, 2)
            assert 0 < t["sweep_ms"] <= t["total_gpu_ms"] + 1e-3
    finally:
        cb.cuboid_enable_timing(g, False)
    ref = oracle.sieve(1, 2000, 1, 2000, primes)
    _cmp(cb.cuboid_sieve_range(g, 1, 2000, 1, 2000, primes), ref)


def test_cache_eviction_keeps_results(pair):
    g, e = pair
    primes = wl.PRIMES_C1
    sizes = [1, 2, 3, 5, 8, 13, 21, 34, 55, 89]     # more shapes than graphs kept
    for rnd in range(2):
        for n in sizes:
            rects = wl.random_rectangles(n, seed=1000 * rnd + n, max_coord=20000, max_side=500)
            st_g, out_g = cb.cuboid_sieve_batch(g, rects, primes, caps=512)
            st_e, out_e = cb.cuboid_sieve_batch(e, rects, primes, caps=512)
            assert st_g == st_e
            _same_batch(out_g, out_e)


def test_capacity_rerun_under_graphs(pair):
    g, e = pair
    rects = [(1, 200, 1, 200), (1, 50, 1, 50), (1, 200, 1, 200)]
    for caps in ([100, 100, 3], [26, 0, 26], [0, 0, 0]):
        st_g, out_g = cb.cuboid_sieve_batch(g, rects, wl.PRIMES_C1, caps=caps)
        st_e, out_e = cb.cuboid_sieve_batch(e, rects, wl.PRIMES_C1, caps=caps)
        assert st_g == st_e
        assert list(out_g.status) == list(out_e.status)
        assert list(out_g.n_survivors) == list(out_e.n_survivors)
        assert np.array_equal(out_g.counts, out_e.counts)


def test_call_by_call_path_against_oracle(pair):
    _, e = pair
    for rect, primes in (((1, 200, 1, 200), wl.PRIMES_C1), ((1, 3000, 1, 2000), wl.PRIMES_C2),
                         ((16777200, 16777300, 5, 400), wl.PRIMES_C2)):
        _cmp(cb.cuboid_sieve_range(e, *rect, primes), oracle.sieve(*rect, primes))
    rects = wl.random_rectangles(30, seed=5, max_coord=4000, max_side=300)
    st, out = cb.cuboid_sieve_batch(e, rects, wl.PRIMES_C2, caps=1024)
    assert st == cb.OK
    for rect, r in zip(rects, out):
        _cmp(r, oracle.sieve(*rect, wl.PRIMES_C2))


def test_graphs_off_and_on_again(pair):
    g, _ = pair
    rect = (1, 200, 1, 200)
    ref = oracle.sieve(*rect, wl.PRIMES_C1)
    cb.cuboid_enable_graphs(g, False)
    try:
        _cmp(cb.cuboid_sieve_range(g, *rect, wl.PRIMES_C1), ref)
    finally:
        cb.cuboid_enable_graphs(g, True)
    _cmp(cb.cuboid_sieve_range(g, *rect, wl.PRIMES_C1), ref)


def test_result_arrays_reused_across_calls(pair):
    g, e = pair
    primes = wl.PRIMES_C1
    held = None
    for seed in range(3):
        rects = wl.random_rectangles(50, seed=300 + seed, max_coord=3000, max_side=300)
        st, held_new = cb.cuboid_sieve_batch(g, rects, primes, caps=128, out=held)
        if held is not None:
            assert held_new is held          # same arrays, overwritten
        held = held_new
        st_e, fresh = cb.cuboid_sieve_batch(e, rects, primes, caps=128)
        assert st == st_e
        _same_batch(held, fresh)


def test_replays_on_a_caller_stream(pair):
    # a torch stream: torch and the library share one HIP runtime
    import torch
    side = torch.cuda.Stream()
    g, e = pair
    primes = wl.PRIMES_C2
    for seed in range(3):
        rects = _batch(700 + seed, 62)
        st_g, out_g = cb.cuboid_sieve_batch(g, rects, primes, caps=64, stream=side)
        st_e, out_e = cb.cuboid_sieve_batch(e, rects, primes, caps=64)
        assert st_g == st_e == cb.OK
        _same_batch(out_g, out_e)
        # the context's own work between replays on the caller's stream
        one = cb.cuboid_sieve_range(g, 3, 900, 7, 1100, primes)
        assert one["n_pairs"] == cb.cuboid_sieve_range(e, 3, 900, 7, 1100, primes)["n_pairs"]
    side.synchronize()
