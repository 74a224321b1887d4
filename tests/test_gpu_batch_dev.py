"""Batched sieve with results left in device memory (cuboid_sieve_batch_dev)
against the host-result batch and the oracle: counts, pair counts and the
sorted survivor list, through graph replays and call-by-call launches, with
a survivor capacity that is too small, and argument errors."""
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


def _host_view(reqs, out):
    """(counts, pairs, [(req, idx), ...]) of a host-result batch."""
    surv = []
    for i in range(len(reqs)):
        s = out[i]["survivors"]
        surv += [(i, int(x)) for x in (s if s is not None else [])]
    return out.counts.astype(np.uint64), np.asarray(out.n_pairs, dtype=np.uint64), surv


@pytest.mark.parametrize("graphs", [True, False])
def test_device_results_equal_host_results(ctx, graphs):
    primes = wl.PRIMES_C1     # survivors in most rectangles
    reqs = wl.random_rectangles(60, seed=31, max_coord=3000, max_side=200) + [(1, 200, 1, 200)]
    cb.cuboid_enable_graphs(ctx, graphs)
    dev = cb.DeviceBatch(ctx, len(reqs), len(primes), surv_cap=1 << 16)
    try:
        st_h, out = cb.cuboid_sieve_batch(ctx, reqs, primes, caps=1 << 14)
        assert st_h == cb.OK
        hc, hp, hs = _host_view(reqs, out)
        for rep in range(3):          # replays reuse the same device buffers
            assert cb.cuboid_sieve_batch_dev(ctx, reqs, primes, dev) == cb.OK
            counts, pairs, surv = dev.read()
            assert np.array_equal(counts, hc)
            assert np.array_equal(pairs, hp)
            assert dev.n_survivors == len(hs)
            assert [(int(e["req"]), int(e["idx"])) for e in surv] == hs
            assert all(int(e["pad"]) == 0 for e in surv)
            # other work on the context between calls
            cb.cuboid_sieve_range(ctx, 5, 300, 7, 400, primes)
    finally:
        dev.free()
        cb.cuboid_enable_graphs(ctx, True)
    # and the oracle for a few of them
    for i in (0, 7, len(reqs) - 1):
        ref = oracle.sieve(*reqs[i], primes)
        assert int(hp[i]) == ref["n_pairs"]
        assert [int(c) for c in hc[i]] == [int(c) for c in ref["counts"]]


def test_device_survivor_capacity(ctx):
    primes = wl.PRIMES_C1
    reqs = [(1, 200, 1, 200), (1, 50, 1, 50), (300, 400, 300, 400)]
    st_h, out = cb.cuboid_sieve_batch(ctx, reqs, primes, caps=1 << 14)
    _, _, hs = _host_view(reqs, out)
    assert len(hs) > 5
    dev = cb.DeviceBatch(ctx, len(reqs), len(primes), surv_cap=5)
    try:
        assert cb.cuboid_sieve_batch_dev(ctx, reqs, primes, dev) == cb.E_CAPACITY
        counts, pairs, surv = dev.read()
        assert dev.n_survivors == len(hs)
        assert [(int(e["req"]), int(e["idx"])) for e in surv] == hs[:5]
        assert np.array_equal(pairs, np.asarray(out.n_pairs, dtype=np.uint64))
    finally:
        dev.free()
    # no survivor buffer at all: counts only
    dev = cb.DeviceBatch(ctx, len(reqs), len(primes), surv_cap=0)
    try:
        assert cb.cuboid_sieve_batch_dev(ctx, reqs, primes, dev) == cb.E_CAPACITY
        assert dev.n_survivors == len(hs)
        counts, _, _ = dev.read()
        assert np.array_equal(counts, out.counts.astype(np.uint64))
    finally:
        dev.free()


def test_device_batch_beyond_resident_rows(ctx):
    primes = wl.PRIMES_C2
    reqs = [(16777000, 16777300, 5, 900), (1, 3000, 1, 2000)]
    dev = cb.DeviceBatch(ctx, len(reqs), len(primes), surv_cap=1 << 12)
    try:
        assert cb.cuboid_sieve_batch_dev(ctx, reqs, primes, dev) == cb.OK
        counts, pairs, surv = dev.read()
    finally:
        dev.free()
    for i, rect in enumerate(reqs):
        ref = oracle.sieve(*rect, primes)
        assert int(pairs[i]) == ref["n_pairs"]
        assert [int(c) for c in counts[i]] == [int(c) for c in ref["counts"]]
        assert [int(e["idx"]) for e in surv if int(e["req"]) == i] == [int(x) for x in ref["survivors"]]


def test_device_batch_errors(ctx):
    primes = wl.PRIMES_C1
    dev = cb.DeviceBatch(ctx, 2, len(primes), surv_cap=4)
    try:
        with pytest.raises(cb.CuboidError) as e:
            cb.cuboid_sieve_batch_dev(ctx, [(1, 10, 1, 10), (0, 5, 1, 5)], primes, dev)
        assert e.value.status == cb.E_RANGE
        d2 = cb.DeviceBatch(ctx, 2, 2)
        try:
            with pytest.raises(cb.CuboidError) as e:
                cb.cuboid_sieve_batch_dev(ctx, [(1, 10, 1, 10), (1, 5, 1, 5)], [4, 7], d2)
            assert e.value.status == cb.E_PRIMES
        finally:
            d2.free()
    finally:
        dev.free()
    with pytest.raises(cb.CuboidError) as e:
        cb.cuboid_device_alloc(ctx, 0)
    assert e.value.status == cb.E_ARG
    cb.cuboid_device_free(ctx, 0)


def test_fresh_context_call_by_call_batches():
    # a context that never captured a graph: its first batches gather counts
    # into buffers allocated during that very call (host and device results)
    primes = wl.PRIMES_C2
    reqs = [(1, 300, 1, 400), (5000, 5100, 20, 3000), (1, 1, 1, 1)]
    h = cb.cuboid_create(0)
    try:
        cb.cuboid_enable_graphs(h, False)
        st, out = cb.cuboid_sieve_batch(h, reqs, primes, caps=1 << 12)
        assert st == cb.OK
        dev = cb.DeviceBatch(h, len(reqs), len(primes), surv_cap=1 << 12)
        try:
            assert cb.cuboid_sieve_batch_dev(h, reqs, primes, dev) == cb.OK
            counts, pairs, surv = dev.read()
        finally:
            dev.free()
    finally:
        assert cb.cuboid_destroy(h) == cb.OK
    for i, rect in enumerate(reqs):
        ref = oracle.sieve(*rect, primes)
        assert out[i]["n_pairs"] == ref["n_pairs"] == int(pairs[i])
        assert [int(c) for c in out[i]["counts"]] == [int(c) for c in ref["counts"]]
        assert [int(c) for c in counts[i]] == [int(c) for c in ref["counts"]]
        assert [int(e["idx"]) for e in surv if int(e["req"]) == i] == [int(x) for x in ref["survivors"]]


@pytest.mark.parametrize("graphs", [True, False])
def test_torch_tensors_on_a_torch_stream(ctx, graphs):
    # results written into torch device tensors (by data_ptr()) on a torch
    # stream other than the default one, behind torch work queued on that
    # stream, against the oracle request by request
    import torch
    primes = wl.PRIMES_C1
    reqs = wl.random_rectangles(40, seed=41, max_coord=3000, max_side=200) + [(1, 200, 1, 200)]
    n, k = len(reqs), len(primes)
    cb.cuboid_enable_graphs(ctx, graphs)
    side = torch.cuda.Stream()
    try:
        with torch.cuda.stream(side):
            # garbage queued on the stream first: the call must come after it
            counts = torch.full((n, k), -1, dtype=torch.int64, device="cuda")
            pairs = torch.full((n,), -1, dtype=torch.int64, device="cuda")
            surv = torch.full((1 << 14, 2), -1, dtype=torch.int64, device="cuda")
            tb = cb.TensorBatch(counts, pairs, surv)
            for rep in range(2):
                assert cb.cuboid_sieve_batch_dev(ctx, reqs, primes, tb, stream=side) == cb.OK
                # torch work after the call on the same stream sees the results
                total = int(pairs.sum().item())
                c, p, s = tb.read()
                assert total == int(p.sum())
                for i, rect in enumerate(reqs):
                    ref = oracle.sieve(*rect, primes)
                    assert int(p[i]) == ref["n_pairs"]
                    assert [int(x) for x in c[i]] == [int(x) for x in ref["counts"]]
                    assert [int(e["idx"]) for e in s if int(e["req"]) == i] == \
                        [int(x) for x in ref["survivors"]]
                counts.fill_(-1)
                pairs.fill_(-1)
        side.synchronize()
    finally:
        cb.cuboid_enable_graphs(ctx, True)


def test_torch_default_stream(ctx):
    import torch
    primes = wl.PRIMES_C2
    reqs = [(1, 3000, 1, 2000), (10**6, 10**6 + 700, 5, 900)]
    counts = torch.zeros((2, len(primes)), dtype=torch.int64, device="cuda")
    pairs = torch.zeros(2, dtype=torch.int64, device="cuda")
    tb = cb.TensorBatch(counts, pairs)
    assert cb.cuboid_sieve_batch_dev(ctx, reqs, primes, tb,
                                     stream=torch.cuda.current_stream()) in (cb.OK, cb.E_CAPACITY)
    c, p, _ = tb.read()
    for i, rect in enumerate(reqs):
        ref = oracle.sieve(*rect, primes)
        assert int(p[i]) == ref["n_pairs"]
        assert [int(x) for x in c[i]] == [int(x) for x in ref["counts"]]


def test_one_hip_runtime():
    # the library and torch share torch's HIP runtime
    import torch  # noqa: F401
    cb.lib()
    assert len(cb.hip_runtimes()) == 1
