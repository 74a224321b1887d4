"""The oracle's stored results at full size against the GPU path:
  * every one of the 4096 rectangles of the batched workload (the
    benchmark's own step, results left in device memory), with the default
    tuning and with the tuning the benchmark runs: per-request counts, pair
    counts and sorted survivor lists;
  * region (1.2) rows at the top of the paper's range (sections 5-6): around
    2^24 (the end of the resident row table), where 59 p crosses 2^31, and
    the last rows below p_max = 72796055 whose q reach 4.29e9, by the region
    sieve (counts, pairs, survivors, r_max per band) and by the background
    search run to the end of the range.
Expected values come from tests/golden/make_golden.py (oracle only).
"""
import json
import os
import time

import numpy as np
import pytest

from paper_1601_00636_amd import binding as cb
from paper_1601_00636_amd import workloads as wl
from tests.conftest import golden_path

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    h = cb.cuboid_create(0)
    yield h
    assert cb.cuboid_destroy(h) == cb.OK


def _say(msg):
    print(msg, flush=True)


def _c4():
    path = golden_path("oracle_c4.npz")
    if not os.path.exists(path):
        pytest.skip("oracle_c4.npz missing")
    return np.load(path)


def _top():
    path = golden_path("oracle_top.json")
    if not os.path.exists(path):
        pytest.skip("oracle_top.json missing")
    with open(path) as f:
        return json.load(f)


@pytest.mark.parametrize("tuned", [False, True])
def test_all_4096_requests_against_the_oracle(ctx, tuned):
    g = _c4()
    reqs = wl.batched_requests(4096)
    primes = [int(r) for r in g["primes"]]
    assert np.array_equal(g["rects"].astype(np.int64), np.asarray(reqs, dtype=np.int64))
    _say("c4 all 4096 requests, tuned=%s" % tuned)
    if tuned:
        cb.cuboid_autotune_for(ctx, primes, reqs)
    dev = cb.DeviceBatch(ctx, len(reqs), len(primes), surv_cap=1 << 16)
    try:
        for rep in range(2):
            st = cb.cuboid_sieve_batch_dev(ctx, reqs, primes, dev)
            assert st == cb.OK
            counts, pairs, surv = dev.read()
            assert np.array_equal(counts, g["counts"])
            assert np.array_equal(pairs, g["n_pairs"])
            g_req = np.repeat(np.arange(len(reqs)), g["n_survivors"].astype(np.int64))
            assert dev.n_survivors == len(g_req)
            assert np.array_equal(surv["req"].astype(np.int64), g_req)
            assert np.array_equal(surv["idx"], g["survivors"])
    finally:
        dev.free()
        cb.cuboid_set_tuning(ctx, primes)


def test_all_4096_requests_host_results(ctx):
    # the same batch with results copied to host memory (cuboid_sieve_batch)
    g = _c4()
    reqs = wl.batched_requests(4096)
    primes = [int(r) for r in g["primes"]]
    st, out = cb.cuboid_sieve_batch(ctx, reqs, primes, caps=64)
    assert st == cb.OK
    assert np.array_equal(out.counts.astype(np.uint64), g["counts"])
    assert np.array_equal(np.asarray(out.n_pairs, dtype=np.uint64), g["n_pairs"])
    off = g["survivor_offsets"].astype(np.int64)
    for i in np.nonzero(g["n_survivors"])[0]:
        assert [int(x) for x in out[int(i)]["survivors"]] == \
            [int(x) for x in g["survivors"][off[i]:off[i + 1]]]


def test_all_4096_requests_served(ctx):
    # the same 4096 rectangles queued on the request server in one call
    # (continuous batching over its launches and streams)
    g = _c4()
    reqs = wl.batched_requests(4096)
    primes = [int(r) for r in g["primes"]]
    off = g["survivor_offsets"].astype(np.int64)
    _say("c4 all 4096 requests through the server")
    srv = cb.cuboid_server_start(ctx, primes, streams=2)
    try:
        tickets = cb.cuboid_server_submit_many(srv, reqs)
        got = [cb.cuboid_server_poll(srv, int(t), len(primes), cap=64) for t in tickets]
        stats = cb.cuboid_server_stats_get(srv)
    finally:
        cb.cuboid_server_stop(srv)
    assert stats["completed"] == len(reqs) and stats["max_admitted"] > 1
    for i, r in enumerate(got):
        assert r["status"] == cb.OK
        assert r["n_pairs"] == int(g["n_pairs"][i])
        assert np.array_equal(np.asarray(r["counts"], dtype=np.uint64), g["counts"][i])
        assert [int(x) for x in r["survivors"]] == [int(x) for x in g["survivors"][off[i]:off[i + 1]]]


def _row_rmax(row, primes):
    if row["n_pairs"] == 0:
        return 1
    if row["n_survivors"]:
        return primes[-1]
    return max(r for r, c in zip(primes, row["counts"]) if c)


def _groups(g):
    rows = g["rows"]
    out = []
    for k in range(0, len(rows), 4):
        out.append(rows[k:k + 4])
    return out


@pytest.mark.parametrize("band", [1, 2, 100])
def test_region_rows_at_the_top_of_the_range(ctx, band):
    g = _top()
    primes = g["primes"]
    for grp in _groups(g):
        p0, p1 = grp[0]["p"], grp[-1]["p"]
        assert [r["p"] for r in grp] == list(range(p0, p1 + 1))
        _say("region rows %d..%d, bands of %d" % (p0, p1, band))
        got = cb.cuboid_sieve_region(ctx, p0, p1, primes, band_rows=band)
        assert got["n_pairs"] == sum(r["n_pairs"] for r in grp)
        assert [int(c) for c in got["counts"]] == \
            [sum(r["counts"][i] for r in grp) for i in range(len(primes))]
        surv = [tuple(x) for r in grp for x in r["survivors"]]
        assert got["n_survivors"] == len(surv)
        assert got["survivors"] == surv
        want = []
        for a in range(0, len(grp), band):
            want.append(max(_row_rmax(r, primes) for r in grp[a:a + band]))
        assert [int(x) for x in got["r_max"]] == want


def test_rectangles_across_the_top_rows(ctx):
    # each top row as a plain rectangle over its region columns: the rectangle
    # path with q up to 4.29e9
    g = _top()
    primes = g["primes"]
    for r in g["rows"]:
        got = cb.cuboid_sieve_range(ctx, r["p"], r["p"], r["qmin"], r["qmax"], primes)
        assert got["n_pairs"] == r["n_pairs"]
        assert [int(c) for c in got["counts"]] == r["counts"]
        assert got["n_survivors"] == r["n_survivors"]


def test_top_rows_through_the_server(ctx):
    # each top row as a rectangle over its region columns, queued on the
    # request server at once: rows beyond the resident row table get their
    # factor lists per request, q reaches 4.29e9
    g = _top()
    primes = g["primes"]
    srv = cb.cuboid_server_start(ctx, primes, streams=2)
    try:
        tickets = cb.cuboid_server_submit_many(
            srv, [(r["p"], r["p"], r["qmin"], r["qmax"]) for r in g["rows"]])
        got = [cb.cuboid_server_poll(srv, int(t), len(primes), cap=1 << 12) for t in tickets]
    finally:
        cb.cuboid_server_stop(srv)
    for r, x in zip(g["rows"], got):
        assert x["status"] == cb.OK
        assert x["n_pairs"] == r["n_pairs"]
        assert [int(c) for c in x["counts"]] == r["counts"]
        assert x["n_survivors"] == r["n_survivors"]


def test_search_runs_to_the_end_of_the_range(ctx):
    # the background search from the first of the last four rows to p_max
    g = _top()
    primes = g["primes"]
    last = [r for r in g["rows"] if r["p"] >= 72796052]
    assert [r["p"] for r in last] == [72796052, 72796053, 72796054, 72796055]
    _say("search from 72796052 to the end")
    h = cb.cuboid_search_start(ctx, primes, 72796052, last[0]["qmin"])
    t0 = time.time()
    while cb.cuboid_search_current(h)["running"]:
        assert time.time() - t0 < 60, "search did not finish"
        time.sleep(0.005)
    found = cb.cuboid_search_survivors(h)
    fin = cb.cuboid_search_stop(h)
    assert fin["status"] == cb.OK
    assert fin["p"] == 72796056 and fin["q"] == 0
    assert fin["pairs"] == sum(r["n_pairs"] for r in last)
    assert fin["survivors"] == sum(r["n_survivors"] for r in last)
    assert found == [tuple(x) for r in last for x in r["survivors"]]
    assert fin["r_max"] == max(_row_rmax(r, primes) for r in last)
