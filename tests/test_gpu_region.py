"""Region (1.2) sieve on the GPU: slices against the oracle, the full scan of
section 6 against the paper's printed result, rows beyond the resident table
against per-row rectangles.
"""
import functools
import json
import os

import numpy as np
import pytest

import oracle
from paper_1601_00636_amd import binding as cb
from paper_1601_00636_amd import workloads as wl
from tests.conftest import golden_path

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    h = cb.cuboid_create(0)
    yield h
    assert cb.cuboid_destroy(h) == cb.OK


def _oracle_band_rmax(p0, p1, band, primes):
    """r_max per band from the oracle's own region sieve of each band."""
    asc = sorted(primes)
    out = []
    for a in range(p0, p1 + 1, band):
        b = min(p1, a + band - 1)
        ref = oracle.sieve_region(a, b, primes)
        if ref["n_pairs"] == 0:
            out.append(1)
        elif ref["n_survivors"]:
            out.append(asc[-1])
        else:
            nz = [asc[i] for i, c in enumerate(ref["counts"]) if c]
            out.append(max(nz))
    return out


def _check_slice(ctx, p0, p1, primes, band):
    ref = oracle.sieve_region(p0, p1, primes)
    got = cb.cuboid_sieve_region(ctx, p0, p1, primes, band_rows=band)
    asc = sorted(primes)
    by_prime = dict(zip(asc, [int(c) for c in ref["counts"]]))
    assert got["n_pairs"] == ref["n_pairs"]
    assert [int(c) for c in got["counts"]] == [by_prime[r] for r in primes]
    assert got["n_survivors"] == ref["n_survivors"]
    assert got["survivors"] == ref["survivors"]
    assert [int(x) for x in got["r_max"]] == _oracle_band_rmax(p0, p1, band, primes)
    return got, ref


@pytest.mark.parametrize("p0,p1,band", [
    (1, 151, 100),       # (5.1): q >= p / 59
    (152, 1151, 100),    # (5.2): q >= cbrt(p / 9), from Start_searching(152, 3)
    (140, 170, 7),       # across the switch between the two lower bounds
    (9000, 9040, 13),
    (40000, 40010, 4),
])
def test_region_slices_against_oracle(ctx, p0, p1, band):
    got, ref = _check_slice(ctx, p0, p1, wl.PRIMES_PAPER, band)
    assert got["n_survivors"] == 0
    depth_prime = wl.PRIMES_PAPER[ref["max_depth"] - 1]
    assert max(int(x) for x in got["r_max"]) == depth_prime


def test_region_survivors_small_primes(ctx):
    # few primes: survivors exist and come back as ascending (p, q)
    primes = [31, 13, 3, 11, 7, 17, 19, 29, 23, 5]
    got, ref = _check_slice(ctx, 1, 300, primes, 50)
    assert got["n_survivors"] > 10
    assert got["survivors"] == sorted(got["survivors"])
    assert max(int(x) for x in got["r_max"]) == 31


@pytest.mark.parametrize("band", [64, 65, 100, 256])
def test_region_bands_split_across_row_blocks(ctx, band):
    # bands of 64 rows or more share row blocks (each lane counts into its own
    # row's band): survivors, totals and every band's r_max against the oracle
    primes = [31, 13, 3, 11, 7, 17, 19, 29, 23, 5]
    got, _ = _check_slice(ctx, 3, 700, primes, band)
    assert got["n_survivors"] > 10
    assert got["survivors"] == sorted(got["survivors"])


def test_region_matches_rectangles_rowwise_beyond_resident_rows(ctx):
    # rows above 2^24 use row windows computed on the fly; each row of the
    # region equals the rectangle [p, p] x [qmin(p), 59 p]
    p0, p1 = 16777213, 16777218
    primes = wl.PRIMES_C2
    got = cb.cuboid_sieve_region(ctx, p0, p1, primes, band_rows=1)
    tot_pairs, tot, surv, rmax = 0, np.zeros(len(primes), dtype=np.int64), [], []
    for p in range(p0, p1 + 1):
        qlo = oracle.region_qmin(p)
        r = cb.cuboid_sieve_range(ctx, p, p, qlo, 59 * p, primes, cap=1 << 12)
        tot_pairs += r["n_pairs"]
        tot += r["counts"].astype(np.int64)
        surv += [(p, qlo + int(i)) for i in r["survivors"]]
        nz = [rp for rp, c in zip(primes, r["counts"]) if c]
        rmax.append(max(primes) if r["n_survivors"] else max(nz))
    assert got["n_pairs"] == tot_pairs
    assert [int(c) for c in got["counts"]] == tot.tolist()
    assert got["survivors"] == surv
    assert [int(x) for x in got["r_max"]] == rmax


def test_region_errors(ctx):
    for args, code in (((0, 5), cb.E_RANGE), ((6, 5), cb.E_RANGE),
                       ((1, 72796056), cb.E_LIMIT)):
        with pytest.raises(cb.CuboidError) as e:
            cb.cuboid_sieve_region(ctx, *args, wl.PRIMES_PAPER)
        assert e.value.status == code
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_sieve_region(ctx, 1, 10, wl.PRIMES_PAPER, band_rows=0)
    assert e.value.status == cb.E_ARG
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_sieve_region(ctx, 1, 300, [11, 13, 17], cap=2)
    assert e.value.status == cb.E_CAPACITY and e.value.needed > 2


def test_section6_scan_matches_the_paper(ctx):
    """p = 1..154000 over region (1.2) with the 96 primes 11..541: the paper
    reports that no pair passes the sieve and that the deepest prime reached is
    the 29th, 137 (section 6)."""
    with open(golden_path("paper_constants.json")) as f:
        pc = json.load(f)
    md = pc["max_depth"]
    primes = wl.PRIMES_PAPER
    assert len(primes) == pc["sieve_primes"]["count"]
    got = cb.cuboid_sieve_region(ctx, 1, md["p_max"], primes, band_rows=100)
    print("section 6 scan: %d coprime pairs, %d survivors, deepest prime %d"
          % (got["n_pairs"], got["n_survivors"], int(got["r_max"].max())), flush=True)
    assert got["n_survivors"] == 0
    assert int(got["r_max"].max()) == md["prime"] == primes[md["index"] - 1]
    assert len(got["r_max"]) == md["p_max"] // 100
    assert sum(int(c) for c in got["counts"]) == got["n_pairs"]
    # the scanned pairs are a coprime subset of the ~0.7e12 the paper counts
    assert 0.55 * pc["pairs_tested"]["value"] < got["n_pairs"] < pc["pairs_tested"]["value"]


def test_section6_scan_against_the_oracle(ctx):
    """The whole scan of section 6 element by element against the oracle's own
    run of it (tests/golden/oracle_s6.json, written by make_golden.py s6):
    per-prime first-rejecter counts, pair count, survivors and r_max for each
    of the 1540 hundreds of p."""
    import os
    path = golden_path("oracle_s6.json")
    if not os.path.exists(path):
        pytest.skip("oracle_s6.json not generated")
    with open(path) as f:
        g = json.load(f)
    got = cb.cuboid_sieve_region(ctx, g["p0"], g["p1"], g["primes"], band_rows=g["band_rows"])
    assert got["n_pairs"] == g["n_pairs"]
    assert [int(c) for c in got["counts"]] == g["counts"]
    assert got["n_survivors"] == g["n_survivors"] == 0
    assert [int(x) for x in got["r_max"]] == g["r_max"]
    assert g["max_depth_prime"] == 137


@functools.lru_cache(maxsize=1)
def _oracle_rows_1_4000():
    ref = oracle.sieve_region(1, 4000, wl.PRIMES_PAPER)
    return ref, _section6_rmax(40) or _oracle_band_rmax(1, 4000, 100, wl.PRIMES_PAPER)


def _section6_rmax(n_bands):
    """r_max of the first bands of 100 rows from the oracle's run of the
    section 6 scan, or None if that file is absent."""
    path = golden_path("oracle_s6.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        g = json.load(f)
    assert g["band_rows"] == 100 and g["primes"] == sorted(wl.PRIMES_PAPER)
    return g["r_max"][:n_bands]


def _region_pairs(p0, p1):
    """Coprime pairs p != q of region (1.2) in rows p0..p1, counted for each
    row by inclusion-exclusion over the prime factors of p."""
    total = 0
    for p in range(p0, p1 + 1):
        lo, hi = oracle.region_qmin(p), 59 * p
        fac, x, d = [], p, 2
        while d * d <= x:
            if x % d == 0:
                fac.append(d)
                while x % d == 0:
                    x //= d
            d += 1
        if x > 1:
            fac.append(x)
        n = 0
        for mask in range(1 << len(fac)):
            m, sign = 1, 1
            for k, f in enumerate(fac):
                if mask >> k & 1:
                    m, sign = m * f, -sign
            n += sign * (hi // m - (lo - 1) // m)
        total += n - (1 if p == 1 and lo <= 1 else 0)
    return total


def test_region_pair_count_formula():
    # the counting formula above against the oracle on a slice
    ref = oracle.sieve_region(1, 300, wl.PRIMES_PAPER)
    assert _region_pairs(1, 300) == ref["n_pairs"]


@pytest.mark.parametrize("schedule", [1, 2, 3])
def test_region_under_each_work_schedule(ctx, schedule):
    # the region scan of rows 1..4000 with primes 11..541 under each way of
    # sharing units between waves, against the oracle
    primes = wl.PRIMES_PAPER
    ref, rmax = _oracle_rows_1_4000()
    cb.cuboid_set_tuning(ctx, primes, schedule=schedule, workgroups=5)
    try:
        got = cb.cuboid_sieve_region(ctx, 1, 4000, primes, band_rows=100)
    finally:
        cb.cuboid_set_tuning(ctx, primes)
    asc = sorted(primes)
    by_prime = dict(zip(asc, [int(c) for c in ref["counts"]]))
    assert got["n_pairs"] == ref["n_pairs"]
    assert [int(c) for c in got["counts"]] == [by_prime[r] for r in primes]
    assert got["survivors"] == ref["survivors"]
    assert [int(x) for x in got["r_max"]] == rmax


def test_region_large_workgroup_pieces(ctx):
    # rows 1..20000 on a grid of one workgroup: over 32 * 4096 units, so the
    # workgroup's share comes in pieces of 4096 units; against round-robin
    # pieces per wave on the full grid, the pair count by inclusion-exclusion
    # and the oracle's r_max of each hundred rows
    primes = wl.PRIMES_PAPER
    cb.cuboid_set_tuning(ctx, primes, schedule=1)
    try:
        ref = cb.cuboid_sieve_region(ctx, 1, 20000, primes, band_rows=100)
        cb.cuboid_set_tuning(ctx, primes, schedule=3, workgroups=1)
        got = cb.cuboid_sieve_region(ctx, 1, 20000, primes, band_rows=100)
    finally:
        cb.cuboid_set_tuning(ctx, primes)
    assert ref["n_pairs"] > 32 * 4096 * 4096 // 2
    assert got["n_pairs"] == ref["n_pairs"] == _region_pairs(1, 20000)
    assert [int(c) for c in got["counts"]] == [int(c) for c in ref["counts"]]
    assert got["survivors"] == ref["survivors"] == []
    assert [int(x) for x in got["r_max"]] == [int(x) for x in ref["r_max"]]
    rmax = _section6_rmax(200)
    if rmax is not None:
        assert [int(x) for x in got["r_max"]] == rmax
