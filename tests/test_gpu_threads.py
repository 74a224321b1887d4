"""Several host threads on one context, and several contexts at once: every
result equals the one the same call gives alone (calls on a context are
serialised; results never depend on concurrency)."""
import threading

import numpy as np
import pytest

from paper_1601_00636_amd import binding as cb
from paper_1601_00636_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _jobs():
    out = []
    for j in range(12):
        rects = wl.random_rectangles(20 + 7 * j, seed=500 + j, max_coord=200000, max_side=1500)
        primes = wl.PRIMES_C2 if j % 3 else wl.PRIMES_BATCHED
        out.append((rects, primes))
    return out


def _run(ctx, job):
    rects, primes = job
    st, res = cb.cuboid_sieve_batch(ctx, rects, primes, caps=64)
    one = cb.cuboid_sieve_range(ctx, *rects[0], primes)
    reg = cb.cuboid_sieve_region(ctx, 3000, 3100, wl.PRIMES_PAPER)
    return (st, res.counts.copy(), np.array(res.n_pairs), np.array(res.n_survivors),
            one["n_pairs"], list(one["counts"]), reg["n_pairs"], list(reg["r_max"]))


def _same(a, b):
    assert a[0] == b[0]
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])
    assert a[4:] == b[4:]


def _threaded(ctxs, jobs):
    got = [None] * len(jobs)
    errs = []

    def work(i):
        try:
            got[i] = _run(ctxs[i % len(ctxs)], jobs[i])
        except Exception as e:        # reported after the join
            errs.append(e)

    ts = [threading.Thread(target=work, args=(i,)) for i in range(len(jobs))]
    for t in ts:
        t.start()
    for t in ts:
        t.join(timeout=120)
    assert not errs, errs
    return got


def test_threads_share_one_context():
    ctx = cb.cuboid_create(0)
    try:
        jobs = _jobs()
        alone = [_run(ctx, j) for j in jobs]
        for _ in range(2):
            for a, b in zip(_threaded([ctx], jobs), alone):
                _same(a, b)
    finally:
        assert cb.cuboid_destroy(ctx) == cb.OK


def test_threads_on_several_contexts():
    ctxs = [cb.cuboid_create(0) for _ in range(3)]
    try:
        jobs = _jobs()
        alone = [_run(ctxs[0], j) for j in jobs]
        for a, b in zip(_threaded(ctxs, jobs), alone):
            _same(a, b)
    finally:
        for c in ctxs:
            assert cb.cuboid_destroy(c) == cb.OK


def test_destroy_while_calls_run():
    # threads loop on one context while another thread destroys it: every
    # call returns OK or E_NOT_LOADED (once the context is gone), destroy
    # returns E_BUSY while a call holds the context, and nothing crashes
    ctx = cb.cuboid_create(0)
    primes = wl.PRIMES_C2
    ref = cb.cuboid_sieve_range(ctx, 1, 700, 1, 900, primes)["n_pairs"]
    seen, errs = [], []
    started = threading.Barrier(5)

    def worker():
        started.wait()
        for _ in range(2000):
            try:
                r = cb.cuboid_sieve_range(ctx, 1, 700, 1, 900, primes)
                if r["n_pairs"] != ref:
                    errs.append(r["n_pairs"])
                seen.append(cb.OK)
            except cb.CuboidError as e:
                seen.append(e.status)
                if e.status != cb.E_NOT_LOADED:
                    errs.append(e)
                return

    ts = [threading.Thread(target=worker) for _ in range(4)]
    for t in ts:
        t.start()
    started.wait()
    busy = 0
    while True:
        st = cb.cuboid_destroy(ctx)
        if st == cb.OK:
            break
        assert st == cb.E_BUSY
        busy += 1
    for t in ts:
        t.join(timeout=120)
    assert not errs, errs
    assert set(seen) <= {cb.OK, cb.E_NOT_LOADED}
    assert cb.cuboid_destroy(ctx) == cb.E_NOT_LOADED


def test_stale_handle_after_a_new_context():
    # a destroyed context's handle stays refused when a new context takes
    # its place (handles carry a generation, not an address)
    old = cb.cuboid_create(0)
    assert cb.cuboid_destroy(old) == cb.OK
    new = cb.cuboid_create(0)
    try:
        assert new.value != old.value
        with pytest.raises(cb.CuboidError) as e:
            cb.cuboid_sieve_range(old, 1, 5, 1, 5, [11])
        assert e.value.status == cb.E_NOT_LOADED
        assert cb.cuboid_destroy(old) == cb.E_NOT_LOADED
        assert cb.cuboid_sieve_range(new, 1, 200, 1, 200, wl.PRIMES_C1)["n_survivors"] == 26
    finally:
        assert cb.cuboid_destroy(new) == cb.OK


def test_servers_and_plain_calls_on_one_context():
    # two request servers with different prime lists and plain calls from
    # other threads share one context at the same time: every result equals
    # the plain call's alone
    ctx = cb.cuboid_create(0)
    try:
        jobs = _jobs()[:6]
        alone = [_run(ctx, j) for j in jobs]
        mix_a = wl.random_rectangles(300, seed=71, max_coord=900000, max_side=3000)
        mix_b = wl.random_rectangles(300, seed=72, max_coord=900000, max_side=3000)
        ref_a = [cb.cuboid_sieve_range(ctx, *r, wl.PRIMES_BATCHED, cap=1 << 14) for r in mix_a]
        ref_b = [cb.cuboid_sieve_range(ctx, *r, wl.PRIMES_C2, cap=1 << 14) for r in mix_b]
        srv_a = cb.cuboid_server_start(ctx, wl.PRIMES_BATCHED, max_launch_units=1 << 12)
        srv_b = cb.cuboid_server_start(ctx, wl.PRIMES_C2, max_launch_units=1 << 12)
        got = [None] * len(jobs)
        errors = []

        def plain(i):
            try:
                got[i] = _run(ctx, jobs[i])
            except Exception as e:   # noqa: BLE001 (reported below)
                errors.append(e)

        try:
            threads = [threading.Thread(target=plain, args=(i,)) for i in range(len(jobs))]
            for t in threads:
                t.start()
            ta = cb.cuboid_server_submit_many(srv_a, mix_a)
            tb = [cb.cuboid_server_submit(srv_b, r) for r in mix_b]
            res_a = [cb.cuboid_server_poll(srv_a, int(t), len(wl.PRIMES_BATCHED), cap=1 << 14)
                     for t in ta]
            res_b = [cb.cuboid_server_poll(srv_b, t, len(wl.PRIMES_C2), cap=1 << 14) for t in tb]
            for t in threads:
                t.join()
        finally:
            cb.cuboid_server_stop(srv_a)
            cb.cuboid_server_stop(srv_b)
        assert not errors, errors
        for a, g in zip(alone, got):
            _same(a, g)
        for ref, x in zip(ref_a + ref_b, res_a + res_b):
            assert x["status"] == cb.OK
            assert x["n_pairs"] == ref["n_pairs"]
            assert [int(c) for c in x["counts"]] == [int(c) for c in ref["counts"]]
            assert [int(s) for s in x["survivors"]] == [int(s) for s in ref["survivors"]]
    finally:
        assert cb.cuboid_destroy(ctx) == cb.OK
