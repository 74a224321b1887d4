#!/usr/bin/env python3
"""Benchmark of the modulo-primes cuboid sieve (arXiv:1601.00636) on one MI355X.

One step = the whole hot path over one batch of synthetic input: the 4096
seeded rectangles of the batched workload (sides log-uniform in [32, 3e4],
origins uniform in [1, 1e6], primes 3 <= r < 500) sieved in one persistent
launch (tables resident, counts and sorted survivors returned per request),
then the exact root check of every survivor.  The value is coprime p != q
pairs per second over the timed steps.

Printed: one JSON line with the metric, a roofline object for the sweep
kernel (HIP-event durations on its stream), the CPU oracle baseline on a
bounded sample, and side measurements (plain launches, the large plain
square).

usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "coprime (p,q) pairs sieved/sec at 1 GPU, bit-exact; batched vs plain; p50/p99"
# 256 CUs x 4 SIMDs x 16 lanes: 64 INT32 lane-operations per clock per CU, at 2.4 GHz
INT32_PEAK = 256 * 64 * 2.4e9
# LDS: 128 bytes per clock per CU
LDS_PEAK = 256 * 128 * 2.4e9
# VALU issue: one wave64 instruction every 4 cycles on each of 1024 SIMDs
SIMDS, CLOCK = 1024, 2.4e9

# Work model of the bit-sliced sweep, per lane and 64-column window (64 pairs
# of one row p):
#   wheel (2, 3, 5): step the window's wheel offset, complement the word   3
#   each prime factor l >= 7 of p: its multiple pattern OR-ed in (2), the
#     pattern index (1), the distance to the next multiple advanced (3)     6
#   coprime-pair count: two 32-bit popcounts                                 2
#   each dense prime: table address (1), AND-NOT (2), two popcounts (2)      5
#   leftover test for the deep path (one 64-bit compare)                     1
# and 10 lane-operations per deep lookup (two residues by multiply-high,
# the inverse and ratio-vector reads, one modular product, the test).
# LDS bytes per lane and window: 8 for the wheel word, 8 per factor >= 7,
# 8 per dense prime.
W_FIXED, W_FACTOR, W_DENSE, W_DEEP = 6, 6, 5, 10


def omega_weighted(rects, least=2):
    """Mean number of distinct prime factors >= least of p over the raw pairs
    of the rectangles (each row weighted by its column count)."""
    pmax = max(r[1] for r in rects)
    is_p = np.ones(pmax + 1, dtype=bool)
    is_p[:2] = False
    for i in range(2, int(pmax**0.5) + 1):
        if is_p[i]:
            is_p[i * i::i] = False
    omega = np.zeros(pmax + 1, dtype=np.int32)
    for ell in np.nonzero(is_p)[0]:
        if ell >= least:
            omega[ell::ell] += 1
    num = den = 0.0
    for p0, p1, q0, q1 in rects:
        w = q1 - q0 + 1
        num += float(omega[p0:p1 + 1].sum()) * w
        den += float(p1 - p0 + 1) * w
    return num / den


def deep_lookups(counts_total, n_surv, primes, trivial, k_dense):
    """Table lookups the deep path makes: every pair that passes the first
    k_dense non-trivial primes is tested against the later ones in ascending
    order until one rejects it (all of them for a survivor)."""
    order = np.argsort(primes)
    k = 0
    tot = 0
    for i in order:
        if trivial[i]:
            continue
        k += 1
        if k > k_dense:
            tot += (k - k_dense) * int(counts_total[i])
    return tot + max(0, k - k_dense) * n_surv


def sweep_work_model(rects, k_dense, deep):
    """(VALU lane-operations, LDS bytes, units) of the work model for one
    sweep over the rectangles: units = raw pairs / 4096, so ragged tiles at
    request edges earn nothing."""
    w7 = omega_weighted(rects, least=7)
    raw = sum((p1 - p0 + 1) * (q1 - q0 + 1) for p0, p1, q0, q1 in rects)
    units = raw / 4096.0
    ops = 64 * units * (W_FIXED + W_FACTOR * w7 + W_DENSE * k_dense) + W_DEEP * deep
    lds = 64 * units * 8 * (1 + w7 + k_dense)
    return ops, lds, units, w7


def _sweep_record(name, k_dense):
    """The record of profiles/<name> taken on this sweep source and on the
    kernel instance (dense-prime count) this launch runs, or None."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    try:
        with open(os.path.join(here, "paper_1601_00636_amd", "csrc", "kernels_sieve.hip"), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
        with open(os.path.join(here, "profiles", name)) as f:
            recs = json.load(f).get("records", [])
    except (OSError, ValueError):
        return None
    for rec in recs:
        if (rec.get("kernel_source_sha256") == sha and
                ("sweep_kernel<%d," % k_dense) in (rec.get("kernel") or "")):
            return rec
    return None


def measured_counters(units_live, sweep_s, k_dense):
    """VALU-issue and LDS-bandwidth fractions of the sweep from the committed
    SQ counter record, only while the sweep kernel's source and instance are
    the ones the counters were taken on: per-unit instruction counts times
    this launch's units over its measured duration."""
    rec = _sweep_record("sweep_counters.json", k_dense)
    if rec is None:
        return None
    pu = rec["per_unit"]
    valu = pu["SQ_INSTS_VALU"] * units_live
    lds_inst = pu["SQ_INSTS_LDS"] * units_live
    out = {"valu_insts_per_unit": pu["SQ_INSTS_VALU"],
           "valu_issue_frac": valu * 4 / (SIMDS * CLOCK * sweep_s),
           "lds_insts_per_unit": pu["SQ_INSTS_LDS"],
           "lds_frac": lds_inst * 512 / sweep_s / LDS_PEAK,
           "source": "profiles/sweep_counters.json (%s)" % rec["kernel"]}
    if pu.get("SQ_ACTIVE_INST_LDS"):
        out["lds_bank_conflict_ratio"] = pu["SQ_LDS_BANK_CONFLICT"] / pu["SQ_ACTIVE_INST_LDS"]
    return out


def mean_depth(counts_total, n_surv, primes, trivial):
    """D: mean number of non-trivial table lookups per coprime pair, primes in
    ascending order with early exit, from the per-prime first-rejecter counts."""
    order = np.argsort(primes)
    k = 0
    tot = 0
    for i in order:
        if trivial[i]:
            continue
        k += 1
        tot += k * int(counts_total[i])
    tot += k * n_surv
    return tot, k


def measured_traffic(k_dense):
    """HBM traffic of the sweep from the committed rocprofv3 counter summary,
    only while the sweep kernel's source and instance are the ones the
    counters were taken on."""
    rec = _sweep_record("sweep_traffic.json", k_dense)
    if rec is None:
        return None, None
    return rec["traffic_GBps"], rec["traffic_bytes_per_launch"]


def verify_against_golden(req_arr, primes, counts, pairs, surv):
    """The last timed step's per-request counts, pair counts and sorted
    survivor lists against the oracle's for the same 4096 rectangles
    (tests/golden/oracle_c4.npz, written by tests/golden/make_golden.py from
    the oracle alone)."""
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "tests", "golden", "oracle_c4.npz")
    if not os.path.exists(path):
        return {"ok": None, "why": "oracle_c4.npz missing"}
    g = np.load(path)
    same_input = (np.array_equal(g["rects"].astype(np.int64), req_arr)
                  and np.array_equal(g["primes"].astype(np.int64), np.asarray(primes)))
    g_req = np.repeat(np.arange(len(g["n_survivors"]), dtype=np.int64),
                      g["n_survivors"].astype(np.int64))
    ok = (same_input and np.array_equal(g["counts"], counts) and np.array_equal(g["n_pairs"], pairs)
          and np.array_equal(g_req, surv["req"].astype(np.int64))
          and np.array_equal(g["survivors"], surv["idx"]))
    return {"ok": bool(ok), "against": "tests/golden/oracle_c4.npz (oracle, all 4096 requests)",
            "requests": int(len(pairs)), "coprime_pairs": int(pairs.sum()),
            "survivors": int(len(surv))}


def run_cpu_baseline(reqs, primes, stride):
    import oracle
    for r in primes:
        oracle.table(r)
    sample = reqs[::stride]
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    t0 = time.time()
    pairs = 0
    for rect in sample:
        pairs += oracle.sieve(*rect, primes, cap=1 << 16, threads=threads)["n_pairs"]
    dt = time.time() - t0
    # one thread, on the first 8 rectangles of the same sample
    t1 = time.time()
    pairs1 = 0
    for rect in sample[:8]:
        pairs1 += oracle.sieve(*rect, primes, cap=1 << 16, threads=1)["n_pairs"]
    dt1 = time.time() - t1
    host = host_cpu()
    model = host.get("Model name", "")
    return dict(value=pairs / dt, unit="coprime pairs/s", cores=threads, kind="oracle",
                sample="every %d%s of the 4096 batched rectangles (%d rectangles, %d coprime "
                       "pairs) in %.1f s; tables excluded"
                       % (stride, {1: "st", 2: "nd", 3: "rd"}.get(stride % 10 if stride % 100 not in
                                                                (11, 12, 13) else 0, "th"),
                          len(sample), pairs, dt),
                single_core={"value": pairs1 / dt1, "sample": "the first 8 of those rectangles "
                             "(%d coprime pairs) in %.1f s" % (pairs1, dt1)},
                cpu_model=model, host=host)


def host_cpu():
    """nproc and the lscpu model line of this host."""
    import subprocess
    info = {"nproc": os.cpu_count()}
    try:
        info["nproc"] = int(subprocess.run(["nproc"], capture_output=True, text=True).stdout)
        for ln in subprocess.run(["lscpu"], capture_output=True, text=True).stdout.splitlines():
            k, _, v = ln.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core",
                             "CPU max MHz"):
                info[k.strip()] = v.strip()
    except (OSError, ValueError):
        pass
    return info


def cpu_squares(c3_stride=32, log=True):
    """The CPU-baseline plan of the three plain squares: the oracle (tables
    built first and excluded) on [1, 200]^2 / 3..31, [1, 1e4]^2 / 3..97 and
    [1, 1e5]^2 / 3..997 in full on all host threads, and on one thread (the
    largest square on one thread over every c3_stride-th row, as a full run
    would take about ten minutes)."""
    import oracle
    from paper_1601_00636_amd import workloads as wl
    out = {"host": host_cpu(), "kind": "oracle", "runs": {}}
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    for name in ("c1", "c2", "c3"):
        p0, p1, q0, q1, primes = wl.square(name)
        t = time.time()
        for r in primes:
            oracle.table(r)
        t_tab = time.time() - t
        t = time.time()
        res = oracle.sieve(p0, p1, q0, q1, primes, cap=1 << 16, threads=threads)
        dt = time.time() - t
        one = {}
        if name != "c3":
            t = time.time()
            r1 = oracle.sieve(p0, p1, q0, q1, primes, cap=1 << 16, threads=1)
            d1 = time.time() - t
            one = {"seconds": d1, "pairs_per_s": r1["n_pairs"] / d1, "sample": "full"}
        else:
            t = time.time()
            n1 = 0
            for row in range(p0, p1 + 1, c3_stride):
                n1 += oracle.sieve(row, row, q0, q1, primes, cap=1 << 16, threads=1)["n_pairs"]
            d1 = time.time() - t
            one = {"seconds": d1, "pairs_per_s": n1 / d1,
                   "sample": "every %dth row (%d coprime pairs)" % (c3_stride, n1)}
        out["runs"][name] = {"n_pairs": int(res["n_pairs"]), "survivors": int(res["n_survivors"]),
                             "tables_seconds": t_tab, "all_threads": {"threads": threads,
                             "seconds": dt, "pairs_per_s": res["n_pairs"] / dt},
                             "one_thread": one}
        if log:
            print(name, json.dumps(out["runs"][name]), file=sys.stderr, flush=True)
    return out


def cpu_full():
    print(json.dumps(cpu_squares()))
    return 0


def calibrate_copy():
    """A plain copy of 2^28 float32 (1 GiB read, 1 GiB written), five times: the
    reference the HBM byte counters of the sweep are scaled by."""
    import torch
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 5
    print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30,
                      "seconds": dt, "GBps_read_plus_write": 2 * (1 << 30) / dt / 1e9}))
    return 0


def replay_to_server(cb, srv, stream, n_primes, cap):
    """Submit a timed stream [(arrival s, rect)] to a server as it arrives: each
    pass of the host loop queues every request already due in one call, so the
    offered rate is not limited by one call per request.  Returns the results
    and each request's latency from its arrival (server completion stamps and
    this loop use the same monotonic clock)."""
    ats = [int(at * 1e9) for at, _ in stream]
    rects = [r for _, r in stream]
    n = len(rects)
    tickets = []
    t0 = time.monotonic_ns()
    i = 0
    while i < n:
        now = time.monotonic_ns() - t0
        j = i
        while j < n and ats[j] <= now:
            j += 1
        if j > i:
            tickets.extend(int(t) for t in cb.cuboid_server_submit_many(srv, rects[i:j]))
            i = j
    t_sub = (time.monotonic_ns() - t0) / 1e9
    out = [cb.cuboid_server_poll(srv, t, n_primes, cap=cap) for t in tickets]
    lat_ms = np.array([x["done_ns"] - (t0 + a) for x, a in zip(out, ats)], dtype=np.float64) / 1e6
    span = (max(x["done_ns"] for x in out) - (t0 + ats[0])) / 1e9
    return out, lat_ms, span, t_sub


def run_served(cb, wl, ctx, primes, seconds):
    """Replay the seeded Poisson stream (2000 requests/s, areas log-uniform in
    [1e3, 1e9]) against the server; latency = completion - arrival."""
    stream = wl.served_stream(duration=seconds, max_requests=int(2000 * seconds))
    srv = cb.cuboid_server_start(ctx, primes)
    try:
        out, lat, span, _ = replay_to_server(cb, srv, stream, len(primes), 4096)
        stats = cb.cuboid_server_stats_get(srv)
    finally:
        cb.cuboid_server_stop(srv)
    pairs = sum(r["n_pairs"] for r in out)
    return {"requests": len(out), "offered_rate_per_s": 2000, "seconds": seconds,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "max_ms": float(lat.max()), "coprime_pairs": pairs,
            "pairs_per_s_over_span": pairs / span, "launches": stats["launches"],
            "max_admitted": stats["max_admitted"]}


def run_served_vs_plain(cb, wl, ctx, primes, rates=(2000, 20000, 200000), n_req=3000):
    """The same seeded Poisson streams (areas log-uniform in [1e3, 1e9]) at
    several offered rates and as a burst, once through the server (continuous
    batching; due requests queued together) and once as one plain
    cuboid_sieve_range call per request from one thread in arrival order;
    latency = completion - arrival for both."""
    out = {}
    for rate in list(rates) + ["burst"]:
        r = 1e9 if rate == "burst" else float(rate)
        stream = wl.served_stream(rate=r, duration=1e9, max_requests=n_req)
        if rate == "burst":
            stream = [(0.0, rect) for _, rect in stream]
        # served: three replays, each on a fresh server; the one with the
        # median throughput is reported
        runs = []
        for _ in range(3):
            srv = cb.cuboid_server_start(ctx, primes)
            try:
                res, lat, span, t_sub = replay_to_server(cb, srv, stream, len(primes), 1 << 14)
                stats = cb.cuboid_server_stats_get(srv)
            finally:
                cb.cuboid_server_stop(srv)
            pairs = sum(x["n_pairs"] for x in res)
            runs.append((pairs / span, res, lat, span, t_sub, stats))
        runs.sort(key=lambda x: x[0])
        _, res, lat, span, t_sub, stats = runs[1]
        pairs = sum(x["n_pairs"] for x in res)
        served = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                  "pairs_per_s": pairs / span, "span_s": span,
                  "submitted_per_s": len(res) / t_sub if t_sub > 0 else None,
                  "launches": stats["launches"], "max_admitted": stats["max_admitted"],
                  "pairs_per_s_of_the_three": [x[0] for x in runs]}
        # plain, one call per request in arrival order
        lat_p = []
        pairs_p = 0
        t0 = time.perf_counter()
        for (at, rect), x in zip(stream, res):
            while time.perf_counter() - t0 < at:
                pass
            g = cb.cuboid_sieve_range(ctx, *rect, primes, cap=1 << 14)
            lat_p.append(time.perf_counter() - t0 - at)
            pairs_p += g["n_pairs"]
            if g["n_pairs"] != x["n_pairs"]:
                raise RuntimeError("served and plain results differ")
        span_p = time.perf_counter() - t0
        lat_p = np.array(lat_p) * 1e3
        plain = {"p50_ms": float(np.percentile(lat_p, 50)), "p99_ms": float(np.percentile(lat_p, 99)),
                 "pairs_per_s": pairs_p / span_p, "span_s": span_p}
        out[str(rate)] = {"requests": len(res), "coprime_pairs": pairs, "served": served,
                          "plain": plain,
                          "served_over_plain_throughput": served["pairs_per_s"] / plain["pairs_per_s"]}
    return out


def section6_scan(cb, wl, ctx, stream, torch):
    """The scan of the paper's section 6: region (1.2), p = 1..154000, the 96
    primes 11..541, the deepest prime used reported per hundred of p."""
    pp = wl.PRIMES_PAPER
    cb.cuboid_sieve_region(ctx, 1, 154000, pp, band_rows=100, stream=stream)
    reps = []
    for _ in range(3):
        t0 = time.perf_counter()
        g6 = cb.cuboid_sieve_region(ctx, 1, 154000, pp, band_rows=100, stream=stream)
        torch.cuda.synchronize()
        reps.append(time.perf_counter() - t0)
    t6 = cb.cuboid_last_timing(ctx)
    dt = float(np.median(reps))
    return {"p_range": [1, 154000], "primes": "11..541 (96)", "band_rows": 100,
            "coprime_pairs": g6["n_pairs"], "survivors": g6["n_survivors"],
            "deepest_prime": int(g6["r_max"].max()), "ms": dt * 1e3, "sweep_ms": t6["sweep_ms"],
            "tuning": cb.cuboid_get_tuning(ctx, pp),
            "value": g6["n_pairs"] / dt, "paper_hours": 4130 / 60.0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--cpu-stride", type=int, default=32)
    ap.add_argument("--served-seconds", type=float, default=10.0)
    ap.add_argument("--tune-cache", default=None,
                    help="JSON-lines file the autotuner reads its choice from, or appends it to "
                         "(lets a profiled run skip the tuning sweeps)")
    ap.add_argument("--section6-only", action="store_true",
                    help="only run the region scan of the paper's section 6 (for profiling)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device-to-device copy (HBM counter calibration)")
    ap.add_argument("--cpu-full", action="store_true",
                    help="only run the oracle on the three plain squares in full, on all host "
                         "threads and on one (the CPU-baseline plan; minutes of host time)")
    args = ap.parse_args()
    if args.calibrate_copy:
        return calibrate_copy()
    if args.cpu_full:
        return cpu_full()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the benchmark runs on exactly one GPU; --gpus %d is not supported "
              "(across GPUs the sieve would shard by bands of rows p)" % args.gpus,
              file=sys.stderr)
        return 2

    import torch
    from paper_1601_00636_amd import binding as cb
    from paper_1601_00636_amd import workloads as wl

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    ctx = cb.cuboid_create(0)
    if args.section6_only:
        cb.cuboid_enable_timing(ctx, True)
        print(json.dumps(section6_scan(cb, wl, ctx, stream, torch)))
        cb.cuboid_destroy(ctx)
        return 0
    reqs = wl.batched_requests(4096)
    primes = wl.PRIMES_BATCHED
    tun = cb.cuboid_autotune_for(ctx, primes, reqs, cache_path=args.tune_cache)
    cb.cuboid_enable_timing(ctx, True)
    _, trivial = cb.cuboid_canonical_primes(primes)
    trivial = np.array([r in (2, 3, 5, 7) for r in primes])

    req_arr = np.asarray(reqs, dtype=np.int64)

    req_u32 = np.ascontiguousarray(req_arr, dtype=np.uint32)
    # results stay in device memory (allocated once, reused from step to step
    # as a serving loop would); only survivors come back, for the root check
    dev = cb.DeviceBatch(ctx, len(reqs), len(primes), surv_cap=1 << 16)

    def survivors_pq(owner, idx):
        # survivor index i of request j is (p - p0_j) * width_j + (q - q0_j)
        width = req_arr[owner, 3] - req_arr[owner, 2] + 1
        return req_arr[owner, 0] + idx // width, req_arr[owner, 2] + idx % width

    def step():
        st = cb.cuboid_sieve_batch_dev(ctx, req_u32, primes, dev, stream=stream)
        if st != cb.OK:
            raise RuntimeError("batch status %d" % st)
        sweep = cb.cuboid_last_timing(ctx)
        ps = qs = []
        if dev.n_survivors:
            surv = cb.cuboid_device_read(ctx, dev.surv,
                                         np.empty(dev.n_survivors, dtype=cb._SURV_DEV_DTYPE))
            ps, qs = survivors_pq(surv["req"].astype(np.int64), surv["idx"].astype(np.int64))
        roots = cb.cuboid_root_check(ctx, ps, qs) if len(ps) else []
        return len(ps), roots, sweep

    held = [None]   # host result arrays reused from step to step

    def step_host():
        # the same batch with every result copied back to host memory
        st, out = cb.cuboid_sieve_batch(ctx, req_u32, primes, caps=256, stream=stream, out=held[0])
        held[0] = out
        if st != cb.OK:
            raise RuntimeError("batch status %d" % st)
        ns = out.n_survivors.astype(np.int64)
        ps = qs = []
        if ns.sum():
            owner = np.repeat(np.arange(len(ns)), ns)
            take = np.concatenate([np.arange(int(out.offsets[j]), int(out.offsets[j]) + int(ns[j]))
                                   for j in np.nonzero(ns)[0]])
            ps, qs = survivors_pq(owner, out.survivors_flat[take].astype(np.int64))
        return cb.cuboid_root_check(ctx, ps, qs) if len(ps) else []

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    sweeps = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        nsurv, roots, tim = step()
        sweeps.append(tim["sweep_ms"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sweep_avg = float(np.mean(sweeps))
    dev_counts, dev_pairs, dev_surv = dev.read()

    n_pairs = int(dev_pairs.sum())
    counts = dev_counts.sum(axis=0)
    value = n_pairs * args.steps / elapsed
    verified = verify_against_golden(req_arr, primes, dev_counts, dev_pairs, dev_surv)
    # the survey's scalar model: 4 D + 3 w + 1 INT32 operations per coprime pair
    lookups, k_nt = mean_depth(counts, nsurv, primes, trivial)
    dbar = lookups / n_pairs
    wbar = omega_weighted(reqs)
    ops_pair = 4 * dbar + 3 * wbar + 1
    scalar_achieved = ops_pair * n_pairs / (sweep_avg * 1e-3)
    # the bit-sliced work model (per unit of 64 x 64 raw pairs)
    k_dense = int(tim["dense_primes"])
    deep = deep_lookups(counts, nsurv, primes, trivial, k_dense)
    m_ops, m_lds, m_units, w7 = sweep_work_model(reqs, k_dense, deep)
    achieved = m_ops / (sweep_avg * 1e-3)
    lds_achieved = m_lds / (sweep_avg * 1e-3)
    traffic_gbps, traffic_bytes = measured_traffic(k_dense)
    ctr = measured_counters(tim["units"], sweep_avg * 1e-3, k_dense)

    res = {
        "metric": METRIC,
        "value": value,
        "unit": "coprime pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (numpy PCG64, seed 20160401)",
        "config": {"workload": "batched: 4096 seeded rectangles, sides log-uniform [32, 3e4], "
                               "origins uniform [1, 1e6], primes 3..499 (94)",
                   "n_requests": 4096, "coprime_pairs_per_step": n_pairs,
                   "survivors_per_step": nsurv, "roots_found": len(roots),
                   "tuning": tun},
        "extras": {},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": INT32_PEAK / 1e12,
                     "unit": "T lane-ops/s (INT32 VALU)", "frac": achieved / INT32_PEAK,
                     "traffic": traffic_gbps,
                     "traffic_unit": "GB/s HBM (FETCH_SIZE, WRITE_SIZE scaled by a 1 GiB copy)",
                     "traffic_bytes_per_launch": traffic_bytes,
                     "kernel": "sweep_kernel", "sweep_ms": sweep_avg,
                     "model": "per lane and 64-column window: %d + %d per factor >= 7 of p + "
                              "%d per dense prime VALU lane-ops, 8 LDS bytes per word read "
                              "(wheel, factors, dense primes); %d lane-ops per deep lookup"
                              % (W_FIXED, W_FACTOR, W_DENSE, W_DEEP),
                     "units_64x64_raw": m_units, "units_64x64_launched": tim["units"],
                     "dense_primes": k_dense, "mean_factors_ge7": w7, "deep_lookups": deep,
                     "lane_ops_per_launch": m_ops,
                     "lds": {"achieved": lds_achieved / 1e12, "peak": LDS_PEAK / 1e12,
                             "unit": "TB/s", "frac": lds_achieved / LDS_PEAK,
                             "bytes_per_launch": m_lds},
                     "counters": ctr,
                     "model_frac": scalar_achieved / INT32_PEAK,
                     "model_frac_note": "the survey's scalar model, 4 D + 3 w + 1 INT32 "
                                        "operations per coprime pair (D = %.4f lookups, w = "
                                        "%.4f factors): the bit-sliced sweep covers 64 pairs "
                                        "per lane operation, so it exceeds 1" % (dbar, wbar)},
        "verified": verified,
    }

    res["config"]["launch"] = {0: "call by call", 1: "hip graph replay",
                               2: "hip graph captured"}[tim["graph"]]
    if not args.no_extras:
        extras = res["extras"]
        # the same batch launched call by call instead of as one graph replay
        cb.cuboid_enable_graphs(ctx, False)
        step()
        torch.cuda.synchronize()
        n_eager = max(3, args.steps // 2)
        t0 = time.perf_counter()
        for _ in range(n_eager):
            step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / n_eager
        cb.cuboid_enable_graphs(ctx, True)
        extras["batched_call_by_call"] = {"value": n_pairs / dt, "ms_per_step": dt * 1e3}
        # the same batch with counts, pair counts and survivors copied back to
        # host memory inside the step (PCIe-inclusive; not the headline value)
        step_host()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n_eager):
            step_host()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / n_eager
        hc = held[0]
        assert np.array_equal(hc.counts.astype(np.uint64), dev_counts)
        assert np.array_equal(np.asarray(hc.n_pairs, dtype=np.uint64), dev_pairs)
        extras["batched_host_results"] = {"value": n_pairs / dt, "ms_per_step": dt * 1e3}
        # plain calls as a caller makes them: no per-call timing events
        cb.cuboid_enable_timing(ctx, False)
        # the same 4096 rectangles as separate plain launches
        t0 = time.perf_counter()
        tot = 0
        for rect in reqs:
            tot += cb.cuboid_sieve_range(ctx, *rect, primes, cap=256, stream=stream)["n_pairs"]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        extras["plain_per_request"] = {"value": tot / dt, "ms": dt * 1e3,
                                       "batched_speedup": (tot / dt) and value / (tot / dt)}
        # the plain square 1..1e5 with primes 3..997 (wall time without the
        # timing events, then one call with them for the sweep's own time)
        p3 = wl.PRIMES_C3
        cb.cuboid_autotune_for(ctx, p3, [(1, 10**5, 1, 10**5)])
        r3 = cb.cuboid_sieve_range(ctx, 1, 10**5, 1, 10**5, p3, stream=stream)
        reps = []
        for _ in range(5):
            t0 = time.perf_counter()
            r3 = cb.cuboid_sieve_range(ctx, 1, 10**5, 1, 10**5, p3, stream=stream)
            torch.cuda.synchronize()
            reps.append(time.perf_counter() - t0)
        cb.cuboid_enable_timing(ctx, True)
        cb.cuboid_sieve_range(ctx, 1, 10**5, 1, 10**5, p3, stream=stream)
        t3 = cb.cuboid_last_timing(ctx)
        cb.cuboid_enable_timing(ctx, False)
        extras["plain_square_1e5"] = {"tuning": cb.cuboid_get_tuning(ctx, p3),
                                      "value": r3["n_pairs"] / float(np.median(reps)),
                                      "ms": float(np.median(reps)) * 1e3,
                                      "sweep_ms": t3["sweep_ms"], "n_pairs": r3["n_pairs"],
                                      "sweep_pairs_per_s": r3["n_pairs"] / (t3["sweep_ms"] * 1e-3)}
        # the two small plain configurations: [1, 200]^2 with 3..31 and
        # [1, 10^4]^2 with 3..97, median of 5 calls each (latency-bound)
        for name, (side, prs) in (("plain_square_200", (200, wl.PRIMES_C1)),
                                  ("plain_square_1e4", (10**4, wl.PRIMES_C2))):
            r = cb.cuboid_sieve_range(ctx, 1, side, 1, side, prs, stream=stream)
            reps = []
            for _ in range(5):
                t0 = time.perf_counter()
                r = cb.cuboid_sieve_range(ctx, 1, side, 1, side, prs, stream=stream)
                reps.append(time.perf_counter() - t0)
            dt = float(np.median(reps))
            extras[name] = {"n_pairs": r["n_pairs"], "survivors": r["n_survivors"],
                            "ms": dt * 1e3, "value": r["n_pairs"] / dt}

    if not args.no_extras:
        cb.cuboid_enable_timing(ctx, True)
        res["extras"]["section6_scan"] = section6_scan(cb, wl, ctx, stream, torch)
        cb.cuboid_enable_timing(ctx, False)
        # the background search of section 5 from Start_searching(152, 3), for
        # about two seconds: pairs sieved per second and how far it got
        h = cb.cuboid_search_start(ctx, wl.PRIMES_PAPER, 152, 3)
        t0 = time.perf_counter()
        time.sleep(2.0)
        rep = cb.cuboid_search_stop(h)
        dt = time.perf_counter() - t0
        res["extras"]["search"] = {"from": [152, 3], "seconds": dt, "exit_p": rep["p"],
                                   "exit_q": rep["q"], "r_max": rep["r_max"],
                                   "coprime_pairs": rep["pairs"], "survivors": rep["survivors"],
                                   "value": rep["pairs"] / dt}
        # the paper's table files for its 96 primes, written and read back
        import tempfile
        with tempfile.TemporaryDirectory() as td:
            tp, pp_ = os.path.join(td, "tables.bin"), os.path.join(td, "primes.bin")
            t0 = time.perf_counter()
            cb.cuboid_write_table_files(ctx, wl.PRIMES_PAPER, tp, pp_)
            t1 = time.perf_counter()
            back = cb.cuboid_check_table_files(ctx, tp, pp_)
            t2 = time.perf_counter()
            res["extras"]["table_files_11_541"] = {
                "primes": len(back), "tables_bytes": os.path.getsize(tp),
                "write_ms": (t1 - t0) * 1e3, "check_ms": (t2 - t1) * 1e3}
        # a deep prime list: the 1193 primes 11..9697 (the paper's format
        # limit) on a 32768 x 32768 square from 10^6
        deep = wl.primes_upto(9697, 11)
        sq = (10**6, 10**6 + 32767, 10**6, 10**6 + 32767)
        rd = cb.cuboid_sieve_range(ctx, *sq, deep, stream=stream)
        t0 = time.perf_counter()
        rd = cb.cuboid_sieve_range(ctx, *sq, deep, stream=stream)
        dt = time.perf_counter() - t0
        res["extras"]["deep_list_9697"] = {"primes": len(deep), "n_pairs": rd["n_pairs"],
                                           "survivors": rd["n_survivors"], "ms": dt * 1e3,
                                           "value": rd["n_pairs"] / dt}
        # measured throughputs of the two units that bound the sweep
        pk = cb.cuboid_probe_peaks(ctx)
        res["extras"]["measured_peaks"] = pk
        res["roofline"]["frac_of_measured_peak"] = achieved / pk["valu_lane_ops_per_s"]
        res["roofline"]["lds"]["frac_of_measured_peak"] = lds_achieved / pk["lds_bytes_per_s"]

    if not args.no_extras and args.served_seconds > 0:
        res["extras"]["served"] = run_served(cb, wl, ctx, primes, args.served_seconds)
        res["extras"]["served_vs_plain"] = run_served_vs_plain(cb, wl, ctx, primes)

    if not args.no_cpu_baseline:
        res["cpu_baseline"] = run_cpu_baseline(reqs, primes, args.cpu_stride)
        # the three plain squares in full (the largest on one thread over
        # every 64th row)
        sq = cpu_squares(c3_stride=64)
        res["cpu_baseline"]["squares"] = sq["runs"]
    dev.free()
    cb.cuboid_destroy(ctx)
    print(json.dumps(res))
    return 0


if __name__ == "__main__":
    sys.exit(main())
