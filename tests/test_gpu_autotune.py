"""Autotuning: the tuning it picks is one of its candidates, results do not
depend on it, a cache file brings the same choice back, and a tuning sample
made of the caller's own requests is validated like a batch."""
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


def _cus(ctx):
    # the default grid is one workgroup per compute unit
    return cb.cuboid_get_tuning(ctx, [11, 13])["workgroups"]


def _same(res, ref):
    assert res["n_pairs"] == ref["n_pairs"]
    assert [int(c) for c in res["counts"]] == [int(c) for c in ref["counts"]]
    assert [int(x) for x in res["survivors"]] == [int(x) for x in ref["survivors"]]


def test_autotune_for_a_sample_and_its_cache(ctx, tmp_path):
    primes = wl.PRIMES_C2
    sample = [(1, 700, 1, 900), (5000, 5100, 20, 30000), (123456, 123999, 7, 77)]
    cache = str(tmp_path / "tune.jsonl")
    t = cb.cuboid_autotune_for(ctx, primes, sample, cache_path=cache)
    cus = _cus(ctx)
    assert t["workgroups"] in (cus, 2 * cus, 4 * cus, 8 * cus)
    assert 0 <= t["dense_primes"] <= 12
    # the work sharing is one of the candidates
    assert (t["schedule"], t["piece_units"]) in {(0, 0), (0, 64), (0, 128), (0, 512), (0, 1024),
                                                 (0, 4096), (1, 0), (1, 64), (2, 0)}
    assert cb.cuboid_get_tuning(ctx, primes)["dense_primes"] == t["dense_primes"]
    for rect in sample:
        _same(cb.cuboid_sieve_range(ctx, *rect, primes, cap=1 << 16),
              oracle.sieve(*rect, primes))
    # a fresh context reads the same choice back from the cache
    other = cb.cuboid_create(0)
    try:
        assert cb.cuboid_autotune_for(other, primes, sample, cache_path=cache) == t
    finally:
        cb.cuboid_destroy(other)
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and "_w3_" in lines[0]     # keyed by the sample too
    assert '"schedule": %d' % t["schedule"] in lines[0]
    assert '"piece_units": %d' % t["piece_units"] in lines[0]
    cb.cuboid_set_tuning(ctx, primes)


def test_autotune_for_rejects_bad_samples(ctx):
    primes = wl.PRIMES_C2
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_autotune_for(ctx, primes, np.zeros((0, 4), dtype=np.uint32))
    assert e.value.status == cb.E_ARG
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_autotune_for(ctx, primes, [(1, 10, 1, 10), (0, 5, 1, 5)])
    assert e.value.status == cb.E_RANGE


def test_autotune_default_sample(ctx):
    primes = [11, 13, 17, 19, 23, 29, 31]
    t = cb.cuboid_autotune(ctx, primes)
    cus = _cus(ctx)
    assert t["workgroups"] in (cus, 2 * cus, 4 * cus, 8 * cus)
    rect = (2, 300, 1, 5000)
    _same(cb.cuboid_sieve_range(ctx, *rect, primes), oracle.sieve(*rect, primes))
    cb.cuboid_set_tuning(ctx, primes)


def test_default_tuning_fills_the_lds(ctx):
    # by default the dense tables take all the LDS a workgroup has left, one
    # workgroup per compute unit
    t = cb.cuboid_get_tuning(ctx, wl.PRIMES_PAPER)
    assert t["workgroups"] == _cus(ctx) > 0
    sizes = [8 * r * (r + 16) for r in wl.PRIMES_PAPER[:13]]
    k = t["dense_primes"]
    assert sum(sizes[:k]) <= t["lds_budget"] < sum(sizes[:k + 1])


def test_cache_lines_without_work_sharing_fields(ctx, tmp_path):
    # a cache line written before the work-sharing fields existed reads back
    # with the defaults
    primes = [11, 13, 17]
    cache = tmp_path / "old.jsonl"
    t = cb.cuboid_autotune(ctx, primes, cache_path=str(cache))
    line = cache.read_text().splitlines()[0]
    old = line.replace(', "schedule": %d, "piece_units": %d' % (t["schedule"], t["piece_units"]), "")
    assert old != line
    cache.write_text(old + "\n")
    other = cb.cuboid_create(0)
    try:
        got = cb.cuboid_autotune(other, primes, cache_path=str(cache))
    finally:
        cb.cuboid_destroy(other)
    assert got["schedule"] == 0 and got["piece_units"] == 0
    assert got["dense_primes"] == t["dense_primes"] and got["workgroups"] == t["workgroups"]
    cb.cuboid_set_tuning(ctx, primes)
