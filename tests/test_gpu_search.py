"""Resumable background search over region (1.2) (section 5's search loop):
what the search scans equals one region sieve (and the oracle) over the same
rows, a stop and a restart from the exit point leave no gap and no overlap,
the report line has the paper's form.
"""
import re
import time

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


def _wait(h, timeout=60.0):
    t0 = time.time()
    while True:
        r = cb.cuboid_search_current(h)
        if not r["running"]:
            return r
        assert time.time() - t0 < timeout, "search did not finish"
        time.sleep(0.005)


def test_search_equals_region_and_oracle(ctx, tmp_path):
    primes = wl.PRIMES_PAPER
    report = tmp_path / "report.txt"
    h = cb.cuboid_search_start(ctx, primes, 152, 3, p_end=2599, report_path=str(report))
    _wait(h)
    fin = cb.cuboid_search_stop(h)
    assert fin["status"] == cb.OK and fin["running"] == 0
    assert fin["p"] == 2600 and fin["q"] == oracle.region_qmin(2600)
    assert fin["p_hundred"] == 2600
    ref = oracle.sieve_region(152, 2599, primes)
    assert fin["pairs"] == ref["n_pairs"]
    assert fin["survivors"] == ref["n_survivors"] == 0
    last = oracle.sieve_region(2500, 2599, primes)
    assert fin["r_max"] == max(r for r, c in zip(sorted(primes), last["counts"]) if c)
    text = report.read_text().splitlines()
    assert re.fullmatch(r"\d{4}-\d{1,2}-\d{1,2} \d{2}:\d{2}", text[0])
    assert text[1] == "Stop with p=2600, q=%d, r_max=%d" % (fin["q"], fin["r_max"])


def test_stop_and_restart_leave_no_gap(ctx):
    primes = wl.PRIMES_PAPER
    h = cb.cuboid_search_start(ctx, primes, 152, 3)
    while cb.cuboid_search_current(h)["p"] < 2000:
        time.sleep(0.002)
    first = cb.cuboid_search_stop(h)
    assert first["status"] == cb.OK and first["p"] >= 2000
    p1, q1 = first["p"], first["q"]
    assert q1 == oracle.region_qmin(p1)
    h = cb.cuboid_search_start(ctx, primes, p1, q1, p_end=p1 + 20000)
    _wait(h)
    second = cb.cuboid_search_stop(h)
    whole = cb.cuboid_sieve_region(ctx, 152, p1 + 20000, primes)
    assert first["pairs"] + second["pairs"] == whole["n_pairs"]
    assert first["survivors"] + second["survivors"] == whole["n_survivors"] == 0
    assert second["p"] == p1 + 20001


def test_partial_first_row_and_survivors(ctx):
    primes = [11, 13, 17, 19, 23, 29, 31]
    p, q, p_end = 200, 500, 430
    h = cb.cuboid_search_start(ctx, primes, p, q, p_end=p_end)
    _wait(h)
    found = cb.cuboid_search_survivors(h)
    fin = cb.cuboid_search_stop(h)
    row = cb.cuboid_sieve_range(ctx, p, p, q, 59 * p, primes)
    rest = cb.cuboid_sieve_region(ctx, p + 1, p_end, primes)
    assert fin["pairs"] == row["n_pairs"] + rest["n_pairs"]
    expect = [(p, q + int(i)) for i in row["survivors"]] + rest["survivors"]
    assert fin["survivors"] == len(expect) > 0
    assert found == expect
    assert fin["r_max"] == 31     # survivors in the last hundred: every prime used


def test_search_errors(ctx):
    pp = wl.PRIMES_PAPER
    for args, code in (((151, 3), cb.E_RANGE), ((72796056, 3000), cb.E_LIMIT),
                       ((152, 2), cb.E_RANGE), ((152, 59 * 152 + 1), cb.E_RANGE)):
        with pytest.raises(cb.CuboidError) as e:
            cb.cuboid_search_start(ctx, pp, *args)
        assert e.value.status == code
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_search_start(ctx, pp, 1000, 20, p_end=999)
    assert e.value.status == cb.E_RANGE
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_search_start(ctx, [12], 152, 3)
    assert e.value.status == cb.E_PRIMES
    h = cb.cuboid_search_start(ctx, pp, 152, 3)
    try:
        with pytest.raises(cb.CuboidError) as e:
            cb.cuboid_search_start(ctx, pp, 152, 3)
        assert e.value.status == cb.E_BUSY           # one search per context
        assert cb.cuboid_destroy(ctx) == cb.E_BUSY   # not while it runs
        # other calls on the context interleave with the search
        r = cb.cuboid_sieve_range(ctx, 1, 200, 1, 200, wl.PRIMES_C1)
        assert r["n_survivors"] == 26
    finally:
        cb.cuboid_search_stop(h)


def test_plain_calls_while_a_search_runs(ctx):
    # a background search and plain calls on the same context at the same
    # time: the search's totals equal the region sieve's, the plain results
    # equal the oracle's
    primes = wl.PRIMES_PAPER
    h = cb.cuboid_search_start(ctx, primes, 152, 3, p_end=20099)
    try:
        rects = [(1, 300, 1, 300), (5000, 5100, 7, 9000), (123456, 123470, 1, 40000)]
        for _ in range(5):
            for rect in rects:
                got = cb.cuboid_sieve_range(ctx, *rect, wl.PRIMES_C2, cap=1 << 16)
                ref = oracle.sieve(*rect, wl.PRIMES_C2, cap=1 << 16)
                assert got["n_pairs"] == ref["n_pairs"]
                assert [int(c) for c in got["counts"]] == [int(c) for c in ref["counts"]]
                assert [int(x) for x in got["survivors"]] == [int(x) for x in ref["survivors"]]
        _wait(h)
    finally:
        fin = cb.cuboid_search_stop(h)
    reg = cb.cuboid_sieve_region(ctx, 152, 20099, primes)
    assert fin["status"] == cb.OK
    assert fin["p"] == 20100
    assert fin["pairs"] == reg["n_pairs"]
    assert fin["survivors"] == reg["n_survivors"]
