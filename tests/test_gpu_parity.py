"""GPU parity: the HIP path (through the C ABI) against the oracle.

Bit-exact for everything (integer work): unsolvability tables byte for byte,
n_pairs, per-prime counts and sorted survivor lists, root lists.
"""
import functools
import json
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1601_00636_amd import binding as cb
from paper_1601_00636_amd import workloads as wl
from tests.conftest import golden_path

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    h = cb.cuboid_create(0)
    yield h
    assert cb.cuboid_destroy(h) == cb.OK


def _golden(name):
    with open(golden_path(name)) as f:
        return json.load(f)


def _cmp(res, ref):
    assert res["n_pairs"] == ref["n_pairs"]
    assert [int(x) for x in res["counts"]] == [int(x) for x in ref["counts"]]
    assert res["n_survivors"] == ref["n_survivors"]
    assert [int(x) for x in res["survivors"]] == [int(x) for x in ref["survivors"]]


# ---------------------------------------------------------------- Q mod r, tables

def test_q_mod_prime_device(ctx):
    rng = np.random.Generator(np.random.PCG64(11))
    n = 4000
    p = rng.integers(0, 2**32, n, dtype=np.uint64)
    q = rng.integers(0, 2**32, n, dtype=np.uint64)
    t = rng.integers(0, 2**32, n, dtype=np.uint64)
    r = rng.integers(2, 65536, n, dtype=np.uint64)
    r[:50] = [2, 3, 5, 7, 11] * 10
    got = cb.cuboid_q_mod_prime(ctx, p, q, t, r)
    ref = [oracle.q_mod_r(int(a), int(b), int(c), int(d)) for a, b, c, d in zip(p, q, t, r)]
    assert got.tolist() == ref


def test_u11_table_against_paper(ctx):
    rows = []
    with open(golden_path("u11_table.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(x) for x in line.split()])
    b = np.frombuffer(cb.cuboid_table_bytes(ctx, 11), dtype=np.uint8)
    bits = np.unpackbits(b, bitorder="little")[:121].reshape(11, 11)
    assert bits.tolist() == rows


@pytest.mark.parametrize("r", wl.primes_upto(200) + [499, 541, 997])
def test_tables_byte_exact(ctx, r):
    assert cb.cuboid_table_bytes(ctx, r) == oracle.pack(r)


def test_large_prime_table_density(ctx):
    # r = 65521 (largest prime below 2^16): no oracle table at this size;
    # check the GPU table's structure (symmetry, zero row/column/diagonal)
    # on sampled rows and its density against ratio-class counting done with
    # the oracle's Q mod r on sampled ratios.
    r = 4099
    b = np.frombuffer(cb.cuboid_table_bytes(ctx, r), dtype=np.uint8)
    u = np.unpackbits(b, bitorder="little")[: r * r].reshape(r, r)
    assert np.array_equal(u, u.T)
    assert u[0].sum() == 0 and u[:, 0].sum() == 0
    assert u[np.arange(r), np.arange(r)].sum() == 0
    rng = np.random.Generator(np.random.PCG64(5))
    for x in rng.integers(1, r, 6):
        unsolv = all(oracle.q_mod_r(int(x), 1, t, r) for t in range(r))
        assert bool(u[x, 1]) == unsolv


# ---------------------------------------------------------------- sieve, full configs

def test_c1_full(ctx):
    g = _golden("oracle_c1.json")
    res = cb.cuboid_sieve_range(ctx, 1, 200, 1, 200, g["primes"])
    _cmp(res, g)


def test_c2_full(ctx):
    g = _golden("oracle_c2.json")
    res = cb.cuboid_sieve_range(ctx, 1, 10**4, 1, 10**4, g["primes"])
    _cmp(res, g)


def test_c3_full(ctx):
    if not os.path.exists(golden_path("oracle_c3.json")):
        pytest.skip("c3 golden missing")
    g = _golden("oracle_c3.json")
    _say("c3 full: 1..1e5 squared, 167 primes")
    res = cb.cuboid_sieve_range(ctx, 1, 10**5, 1, 10**5, g["primes"])
    _cmp(res, g)


# ---------------------------------------------------------------- sieve, random and edges

def test_random_rectangles(ctx):
    rects = wl.random_rectangles(60, seed=123, max_coord=3000, max_side=260)
    rng = np.random.Generator(np.random.PCG64(9))
    pool = wl.primes_upto(300)
    for i, rect in enumerate(rects):
        k = int(rng.integers(1, 30))
        primes = [int(x) for x in rng.choice(pool, size=k, replace=False)]
        ref = oracle.sieve(*rect, primes)
        res = cb.cuboid_sieve_range(ctx, *rect, primes)
        _cmp(res, ref)


@pytest.mark.parametrize("rect", [
    (1, 1, 1, 1), (1, 1, 1, 500), (1, 500, 1, 1), (7, 7, 1, 1000), (1, 64, 1, 64),
    (1, 65, 1, 65), (63, 129, 63, 129), (100, 100, 100, 100), (2, 2, 2, 2),
    (4294967195, 4294967295, 4294967000, 4294967295),
    (4294967295, 4294967295, 1, 300),
    (16777200, 16777300, 5, 400),
    (999983, 1000100, 999900, 1000050),
])
def test_edge_rectangles(ctx, rect):
    primes = wl.PRIMES_C2
    ref = oracle.sieve(*rect, primes)
    res = cb.cuboid_sieve_range(ctx, *rect, primes)
    _cmp(res, ref)


@pytest.mark.parametrize("primes", [wl.PRIMES_C2, [11, 13, 17, 19, 23, 29, 31, 37, 41, 43]])
def test_long_rows(ctx, primes):
    # few row blocks, a million columns: each wave walks thousands of windows
    # of the same rows, through every fold-back of the dense tables' offsets
    rect = (1, 128, 1, 10**6)
    ref = oracle.sieve(*rect, primes)
    for k in (0, 5, 10):
        cb.cuboid_set_tuning(ctx, primes, dense_primes=k, workgroups=4, lds_budget=160 * 1024)
        try:
            res = cb.cuboid_sieve_range(ctx, *rect, primes)
        finally:
            cb.cuboid_set_tuning(ctx, primes)
        _cmp(res, ref)


@pytest.mark.parametrize("rect", [
    (4294967291, 4294967291, 4294900000, 4294967295),   # the largest prime below 2^32
    (4294967279, 4294967291, 4294960000, 4294967295),
    (2147483659, 2147483659, 2147400000, 2147500000),   # a prime just above 2^31
])
def test_prime_rows_above_2_31(ctx, rect):
    # rows whose own prime factor exceeds 2^31, over thousands of windows:
    # the distance to the next multiple of p must wrap without overflowing,
    # so that exactly the column q = p drops out as not coprime
    primes = wl.PRIMES_C2
    ref = oracle.sieve(*rect, primes)
    for wg in (0, 1):
        cb.cuboid_set_tuning(ctx, primes, workgroups=wg)
        try:
            res = cb.cuboid_sieve_range(ctx, *rect, primes, cap=1 << 16)
        finally:
            cb.cuboid_set_tuning(ctx, primes)
        _cmp(res, ref)


@pytest.mark.parametrize("k", [0, 1, 3, 5, 7, 9, 12])
def test_dense_count_does_not_change_results(ctx, k):
    primes = wl.primes_upto(120, 3)
    rect = (3, 700, 11, 900)
    ref = oracle.sieve(*rect, primes)
    cb.cuboid_set_tuning(ctx, primes, dense_primes=k, lds_budget=160 * 1024)
    try:
        res = cb.cuboid_sieve_range(ctx, *rect, primes)
    finally:
        cb.cuboid_set_tuning(ctx, primes)
    _cmp(res, ref)


def test_workgroup_count_does_not_change_results(ctx):
    primes = wl.PRIMES_C2
    rect = (1, 3000, 1, 2000)
    ref = oracle.sieve(*rect, primes)
    for wg in (1, 7, 64, 1000):
        cb.cuboid_set_tuning(ctx, primes, workgroups=wg)
        try:
            res = cb.cuboid_sieve_range(ctx, *rect, primes)
        finally:
            cb.cuboid_set_tuning(ctx, primes)
        _cmp(res, ref)


def test_trivial_and_unsorted_primes(ctx):
    primes = [13, 2, 7, 11, 3, 31, 5]
    ref = oracle.sieve(1, 400, 1, 400, primes)
    res = cb.cuboid_sieve_range(ctx, 1, 400, 1, 400, primes)
    _cmp(res, ref)
    assert res["counts"][1] == res["counts"][2] == res["counts"][4] == res["counts"][6] == 0


def test_only_trivial_primes_all_survive(ctx):
    rect = (1, 90, 1, 80)
    ref = oracle.sieve(*rect, [3, 5, 7])
    res = cb.cuboid_sieve_range(ctx, *rect, [3, 5, 7], cap=10000)
    _cmp(res, ref)
    assert res["n_survivors"] == res["n_pairs"]


def test_paper_primes_region_slice(ctx):
    # the paper's 96 primes 11..541 on a rectangle inside region (1.2)
    rect = (152, 1151, 3, 5000)
    ref = oracle.sieve(*rect, wl.PRIMES_PAPER)
    res = cb.cuboid_sieve_range(ctx, *rect, wl.PRIMES_PAPER)
    _cmp(res, ref)


# ---------------------------------------------------------------- errors

def test_error_codes(ctx):
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_sieve_range(ctx, 0, 5, 1, 5, [11])
    assert e.value.status == cb.E_RANGE
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_sieve_range(ctx, 6, 5, 1, 5, [11])
    assert e.value.status == cb.E_RANGE
    for bad in ([9], [11, 11], [65537], [], [1]):
        with pytest.raises(cb.CuboidError) as e:
            cb.cuboid_sieve_range(ctx, 1, 5, 1, 5, bad)
        assert e.value.status == cb.E_PRIMES
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_sieve_range(ctx, 1, 200, 1, 200, wl.PRIMES_C1, cap=5)
    assert e.value.status == cb.E_CAPACITY and e.value.needed == 26
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_table_bytes(ctx, 12)
    assert e.value.status == cb.E_PRIMES


def test_destroyed_context_is_refused():
    h = cb.cuboid_create(0)
    assert cb.cuboid_destroy(h) == cb.OK
    assert cb.cuboid_destroy(h) == cb.E_NOT_LOADED
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_sieve_range(h, 1, 5, 1, 5, [11])
    assert e.value.status == cb.E_NOT_LOADED


# ---------------------------------------------------------------- root check

def test_root_check_survivors_c1_c2(ctx):
    for name, side in (("oracle_c1.json", 200), ("oracle_c2.json", 10**4)):
        g = _golden(name)
        p = [1 + i // side for i in g["survivors"]]
        q = [1 + i % side for i in g["survivors"]]
        got = cb.cuboid_root_check(ctx, p, q)
        assert [tuple(x[:4]) for x in got] == [tuple(x) for x in g["roots"]] == []


def test_root_check_degenerate_pairs(ctx):
    pairs = [(1, 1), (12, 12), (97, 0), (0, 97), (0, 0), (65536, 65536), (2**31 - 1, 0),
             (30030, 30030), (3, 5), (7, 7)]
    p = [a for a, _ in pairs]
    q = [b for _, b in pairs]
    got = cb.cuboid_root_check(ctx, p, q)
    ref = oracle.root_check(pairs)
    assert [tuple(x[:4]) for x in got] == [tuple(x) for x in ref]
    # p = q gives the root t = p^2 (Q_pp = -(p^2 - t)(p^2 + t)(p^4 + t^2)^4)
    assert (12, 12, 144) in [tuple(x[:3]) for x in got]


def test_root_check_whole_u32_domain(ctx):
    # coordinates up to 2^32 - 1, the sieve's own range (q = 59 p reaches
    # 4.29e9 at the paper's p_max): the root bound on t passes 2^64 there, so
    # candidates are 128-bit; roots p^2 for p = q and q = 0 (eq. 1.1)
    rng = np.random.Generator(np.random.PCG64(11))
    pairs = [(2**32 - 1, 2**32 - 1), (2**32 - 1, 0), (0, 2**32 - 1), (2**31, 0), (2**31, 2**31),
             (3000000019, 3000000019), (4294967291, 4294967279), (2**32 - 1, 1), (1, 2**32 - 1),
             (72796055, 4294967245), (36398028, 2147483652), (2**31 - 1, 2**31 + 1)]
    p = rng.integers(2**31, 2**32, 40)
    q = rng.integers(2**31, 2**32, 40)
    p[:6] = q[:6]   # six more with a root
    pairs += list(zip(p.tolist(), q.tolist()))
    got = cb.cuboid_root_check(ctx, [a for a, _ in pairs], [b for _, b in pairs])
    ref = oracle.root_check(pairs)
    assert [tuple(x[:4]) for x in got] == [tuple(x) for x in ref]
    assert (2**32 - 1, 2**32 - 1, (2**32 - 1)**2) in [tuple(x[:3]) for x in got]
    assert len(got) >= 11   # at least the p = q and (p, 0) pairs


def test_root_check_random_pairs(ctx):
    rng = np.random.Generator(np.random.PCG64(3))
    p = rng.integers(1, 3000, 300)
    q = rng.integers(1, 3000, 300)
    p[:40] = q[:40]   # forty pairs with a root
    got = cb.cuboid_root_check(ctx, p, q)
    ref = oracle.root_check(list(zip(p.tolist(), q.tolist())))
    assert [tuple(x[:4]) for x in got] == [tuple(x) for x in ref]


# ---------------------------------------------------------------- batched

def test_batch_equals_plain(ctx):
    rects = wl.random_rectangles(40, seed=77, max_coord=5000, max_side=400)
    rects += [(1, 200, 1, 200), (10, 10, 20, 20), (1, 1, 1, 1)]
    primes = wl.PRIMES_C2
    st, out = cb.cuboid_sieve_batch(ctx, rects, primes, caps=4096)
    assert st == cb.OK
    for rect, r in zip(rects, out):
        ref = cb.cuboid_sieve_range(ctx, *rect, primes)
        assert r["status"] == cb.OK
        _cmp(r, ref)
        _cmp(r, oracle.sieve(*rect, primes))


def test_batch_capacity_per_request(ctx):
    rects = [(1, 200, 1, 200), (1, 50, 1, 50), (1, 200, 1, 200)]
    st, out = cb.cuboid_sieve_batch(ctx, rects, wl.PRIMES_C1, caps=[100, 100, 3])
    assert st == cb.E_CAPACITY
    assert out[0]["status"] == cb.OK and out[0]["n_survivors"] == 26
    assert out[2]["status"] == cb.E_CAPACITY and out[2]["n_survivors"] == 26
    _cmp(out[0], oracle.sieve(1, 200, 1, 200, wl.PRIMES_C1))


def _coprime_pairs_square(n):
    """Ordered coprime pairs p != q in [1, n]^2: 2 (phi(1) + ... + phi(n)) - 2
    (the diagonal holds only (1, 1))."""
    phi = np.arange(n + 1, dtype=np.int64)
    for k in range(2, n + 1):
        if phi[k] == k:
            phi[k::k] -= phi[k::k] // k
    return 2 * int(phi[1:].sum()) - 2


def test_survivors_beyond_the_device_list(ctx):
    # only trivial primes, so every coprime pair survives: 6.83e7 of them are
    # more than the 2^26 survivors a call keeps on the device, so the call
    # returns E_LIMIT and each request its survivor count (pairs minus the
    # counts) without a list
    n = 10600
    want = _coprime_pairs_square(n)
    assert want > 1 << 26
    primes = [3, 5, 7]
    st, out = cb.cuboid_sieve_batch(ctx, [(1, n, 1, n), (1, 30, 1, 30)], primes, caps=16)
    assert st == cb.E_LIMIT
    assert out[0]["n_pairs"] == want and out[0]["n_survivors"] == want
    assert out[0]["status"] == cb.E_CAPACITY
    assert out[1]["n_pairs"] == out[1]["n_survivors"] == _coprime_pairs_square(30)
    assert out[1]["status"] == cb.E_CAPACITY
    assert [int(c) for c in out[0]["counts"]] == [0, 0, 0]
    dev = cb.DeviceBatch(ctx, 1, len(primes), surv_cap=16)
    try:
        assert cb.cuboid_sieve_batch_dev(ctx, [(1, n, 1, n)], primes, dev) == cb.E_LIMIT
        assert dev.n_survivors == want
        counts, pairs, _ = dev.read()
        assert int(pairs[0]) == want and int(counts.sum()) == 0
    finally:
        dev.free()


@pytest.mark.parametrize("tuned", [False, True])
def test_c4_sample_against_oracle(ctx, tuned):
    # the full 4096-rectangle batch, with the default tuning and with the one
    # the benchmark runs (tuned on the same rectangles), sampled requests
    # against the oracle's
    if not os.path.exists(golden_path("oracle_c4s.json")):
        pytest.skip("c4 sample golden missing")
    g = _golden("oracle_c4s.json")
    reqs = wl.batched_requests(4096)
    _say("c4: 4096 rectangles in one batch, tuned=%s" % tuned)
    if tuned:
        cb.cuboid_autotune_for(ctx, g["primes"], reqs)
    dev = cb.DeviceBatch(ctx, len(reqs), len(g["primes"]), surv_cap=1 << 16)
    try:
        st, out = cb.cuboid_sieve_batch(ctx, reqs, g["primes"], caps=64)
        # the benchmark's own step: results left in device memory
        st_dev = cb.cuboid_sieve_batch_dev(ctx, reqs, g["primes"], dev)
        counts, pairs, surv = dev.read()
    finally:
        dev.free()
        cb.cuboid_set_tuning(ctx, g["primes"])
    assert st == cb.OK and st_dev == cb.OK
    for ref in g["results"]:
        i = ref["index"]
        _cmp(out[i], ref)
        assert int(pairs[i]) == ref["n_pairs"]
        assert [int(c) for c in counts[i]] == [int(c) for c in ref["counts"]]
        assert [int(e["idx"]) for e in surv if int(e["req"]) == i] == [int(x) for x in ref["survivors"]]
    assert np.array_equal(counts, out.counts.astype(np.uint64))


# ---------------------------------------------------------------- work sharing

@pytest.mark.parametrize("schedule", [1, 2, 3])
@pytest.mark.parametrize("wg", [0, 1, 3])
def test_work_schedules(ctx, schedule, wg):
    # round-robin pieces per wave, the shared counter and workgroup pieces
    # (on grids of one, three and all workgroups) give the oracle's results:
    # one rectangle, a batch of many, rows beyond the resident table (one
    # launch per row window, each with its own counter and cursors) and long rows
    primes = wl.PRIMES_C2
    cb.cuboid_set_tuning(ctx, primes, workgroups=wg, schedule=schedule)
    try:
        for rect in ((1, 3000, 1, 2000), (16777000, 16777300, 5, 900), (1, 70, 1, 300000)):
            _cmp(cb.cuboid_sieve_range(ctx, *rect, primes, cap=1 << 16), oracle.sieve(*rect, primes))
        rects = wl.random_rectangles(40, seed=77, max_coord=50000, max_side=700)
        st, out = cb.cuboid_sieve_batch(ctx, rects, primes, caps=4096)
        assert st == cb.OK
        for rect, r in zip(rects, out):
            _cmp(r, oracle.sieve(*rect, primes))
    finally:
        cb.cuboid_set_tuning(ctx, primes)


@pytest.mark.parametrize("wg", [1, 7])
def test_workgroup_pieces_large_and_odd_grids(ctx, wg):
    # 129 row blocks x 1094 windows: on one workgroup more than 32 x 4096 units,
    # so its share comes in pieces of 4096 units; on seven workgroups pieces of
    # 256 units that do not divide evenly between them.  Against round-robin
    # pieces per wave on the full grid.
    primes = wl.PRIMES_C2
    rect = (1, 8200, 1, 70000)
    ref = _oracle_large_rect()
    cb.cuboid_set_tuning(ctx, primes, schedule=1)
    try:
        _cmp(cb.cuboid_sieve_range(ctx, *rect, primes, cap=1 << 16), ref)
        cb.cuboid_set_tuning(ctx, primes, schedule=3, workgroups=wg)
        got = cb.cuboid_sieve_range(ctx, *rect, primes, cap=1 << 16)
    finally:
        cb.cuboid_set_tuning(ctx, primes)
    assert ref["n_pairs"] > 0
    _cmp(got, ref)


@functools.lru_cache(maxsize=1)
def _oracle_large_rect():
    return oracle.sieve(1, 8200, 1, 70000, wl.PRIMES_C2, cap=1 << 16)


def test_schedule_out_of_range(ctx):
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_set_tuning(ctx, wl.PRIMES_C2, schedule=4)
    assert e.value.status == cb.E_ARG
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_set_tuning(ctx, wl.PRIMES_C2, piece_units=(1 << 20) + 1)
    assert e.value.status == cb.E_ARG


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("piece", [1, 7, 64, 4096, 1 << 20])
def test_piece_sizes(ctx, schedule, piece):
    # every piece size the tuning allows gives the oracle's results, from one
    # unit per piece to pieces larger than the whole launch
    primes = wl.PRIMES_C2
    cb.cuboid_set_tuning(ctx, primes, schedule=schedule, piece_units=piece)
    try:
        assert cb.cuboid_get_tuning(ctx, primes)["piece_units"] == piece
        for rect in ((1, 3000, 1, 2000), (1, 70, 1, 300000)):
            _cmp(cb.cuboid_sieve_range(ctx, *rect, primes, cap=1 << 16), oracle.sieve(*rect, primes))
        rects = wl.random_rectangles(30, seed=91, max_coord=50000, max_side=700)
        st, out = cb.cuboid_sieve_batch(ctx, rects, primes, caps=4096)
        assert st == cb.OK
        for rect, r in zip(rects, out):
            _cmp(r, oracle.sieve(*rect, primes))
    finally:
        cb.cuboid_set_tuning(ctx, primes)
