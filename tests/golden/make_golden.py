"""Writes the oracle's expected values for the rectangle workloads into
tests/golden/oracle_<name>.json.  Calls only the oracle package.

Workloads (sieve over all coprime p != q in the square, primes as listed):
  c1  1 <= p, q <= 200,    primes 3..31
  c2  1 <= p, q <= 10^4,   primes 3..97
  c3  1 <= p, q <= 10^5,   primes 3..997
  c4s a seeded sample of the batched workload's rectangles, primes 3..499
  c4  every one of the batched workload's 4096 rectangles, primes 3..499
      (oracle_c4.npz: per-request counts, pair counts and survivors)
  top region (1.2) row by row, primes 11..541, at three places of the paper's
      range (sec. 5-6): rows around 2^24, the rows where 59 p crosses 2^31,
      and the last rows below p_max = floor(2^32 / 59) = 72796055, whose q
      reach 4.29e9 (oracle_top.json: per-row counts, pair counts, survivors
      and deepest first rejecter)
  s6  region (1.2) for p = 1..154000, primes 11..541 (the scan of section 6),
      per hundred of p: the deepest prime some pair was tested against

usage: python tests/golden/make_golden.py [c1 c2 c3 c4s c4 top s6] [--threads N]
"""
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402


def primes_in(lo, hi):
    return [r for r in range(max(2, lo), hi + 1) if all(r % d for d in range(2, int(r**0.5) + 1))]


SQUARES = {
    "c1": (200, primes_in(3, 31)),
    "c2": (10**4, primes_in(3, 97)),
    "c3": (10**5, primes_in(3, 997)),
}


def square(name):
    n, primes = SQUARES[name]
    t = time.time()
    for r in primes:
        oracle.table(r)
    t_tab = time.time() - t
    t = time.time()
    res = oracle.sieve(1, n, 1, n, primes, cap=1 << 20)
    t_sieve = time.time() - t
    surv = [int(x) for x in res["survivors"]]
    roots = oracle.root_check([(1 + i // n, 1 + i % n) for i in surv])
    out = dict(workload=name, p0=1, p1=n, q0=1, q1=n, primes=primes,
               counts=[int(c) for c in res["counts"]], n_pairs=int(res["n_pairs"]),
               n_survivors=int(res["n_survivors"]), survivors=surv,
               roots=[list(x) for x in roots],
               oracle_seconds=dict(tables=round(t_tab, 2), sieve=round(t_sieve, 2)))
    with open(os.path.join(HERE, "oracle_%s.json" % name), "w") as f:
        json.dump(out, f, indent=1)
    print(name, "pairs", out["n_pairs"], "survivors", out["n_survivors"], out["oracle_seconds"])


def c4_sample():
    sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
    from paper_1601_00636_amd.workloads import batched_requests, PRIMES_BATCHED
    reqs = batched_requests(4096)
    # every 64th request of the seeded batch: 64 rectangles
    picks = list(range(0, 4096, 64))
    out = dict(workload="c4s", primes=PRIMES_BATCHED, picks=picks, results=[])
    t = time.time()
    for i in picks:
        p0, p1, q0, q1 = reqs[i]
        res = oracle.sieve(p0, p1, q0, q1, PRIMES_BATCHED, cap=1 << 16)
        out["results"].append(dict(index=i, rect=[p0, p1, q0, q1],
                                   counts=[int(c) for c in res["counts"]],
                                   n_pairs=int(res["n_pairs"]),
                                   n_survivors=int(res["n_survivors"]),
                                   survivors=[int(x) for x in res["survivors"]]))
    out["oracle_seconds"] = round(time.time() - t, 2)
    with open(os.path.join(HERE, "oracle_c4s.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("c4s", len(picks), "requests", out["oracle_seconds"], "s")


def c4_full(threads=0):
    from paper_1601_00636_amd.workloads import batched_requests, PRIMES_BATCHED
    reqs = batched_requests(4096)
    for r in PRIMES_BATCHED:
        oracle.table(r)
    n, k = len(reqs), len(PRIMES_BATCHED)
    counts = np.zeros((n, k), dtype=np.uint64)
    pairs = np.zeros(n, dtype=np.uint64)
    nsurv = np.zeros(n, dtype=np.uint64)
    surv = []
    t = time.time()
    for i, (p0, p1, q0, q1) in enumerate(reqs):
        res = oracle.sieve(p0, p1, q0, q1, PRIMES_BATCHED, cap=1 << 16, threads=threads)
        assert res["n_survivors"] <= 1 << 16
        counts[i] = res["counts"]
        pairs[i] = res["n_pairs"]
        nsurv[i] = res["n_survivors"]
        surv.append(np.asarray(res["survivors"], dtype=np.uint64))
        if i % 256 == 255:
            print("c4 %d requests: %.0f s" % (i + 1, time.time() - t), flush=True)
    offsets = np.zeros(n + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(nsurv)
    np.savez_compressed(os.path.join(HERE, "oracle_c4.npz"),
                        rects=np.array(reqs, dtype=np.uint64),
                        primes=np.array(PRIMES_BATCHED, dtype=np.uint32),
                        counts=counts, n_pairs=pairs, n_survivors=nsurv,
                        survivor_offsets=offsets,
                        survivors=np.concatenate(surv) if surv else np.zeros(0, np.uint64),
                        oracle_seconds=np.array(time.time() - t))
    print("c4 pairs", int(pairs.sum()), "survivors", int(nsurv.sum()),
          "%.0f s" % (time.time() - t))


# region rows at the top of the paper's range: around 2^24, where 59 p crosses
# 2^31 (2^31 / 59 = 36398027.1...), and the last rows below p_max
TOP_ROWS = (list(range(16777214, 16777218)) + list(range(36398026, 36398030))
            + list(range(72796052, 72796056)))


def top_rows(workers=6):
    primes = primes_in(11, 541)
    for r in primes:
        oracle.table(r)
    t = time.time()

    def one(p):
        res = oracle.sieve_region(p, p, primes, threads=1)
        print("top row %d: %d pairs, %.0f s" % (p, res["n_pairs"], time.time() - t), flush=True)
        return dict(p=p, qmin=oracle.region_qmin(p), qmax=59 * p,
                    counts=[int(c) for c in res["counts"]], n_pairs=int(res["n_pairs"]),
                    n_survivors=int(res["n_survivors"]),
                    survivors=[list(x) for x in res["survivors"]],
                    max_depth=int(res["max_depth"]))
    # the longest rows first
    order = sorted(TOP_ROWS, reverse=True)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        rows = dict(zip(order, ex.map(one, order)))
    out = dict(workload="top", primes=primes, rows=[rows[p] for p in TOP_ROWS],
               oracle_seconds=round(time.time() - t, 1))
    with open(os.path.join(HERE, "oracle_top.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("top", len(TOP_ROWS), "rows", out["oracle_seconds"], "s")


def section6(p_max=154000, band=100):
    primes = primes_in(11, 541)
    for r in primes:
        oracle.table(r)
    counts = [0] * len(primes)
    pairs = surv = 0
    r_max = []
    t = time.time()
    for a in range(1, p_max + 1, band):
        b = min(p_max, a + band - 1)
        res = oracle.sieve_region(a, b, primes)
        pairs += int(res["n_pairs"])
        surv += int(res["n_survivors"])
        cs = [int(c) for c in res["counts"]]
        counts = [x + y for x, y in zip(counts, cs)]
        if res["n_pairs"] == 0:
            r_max.append(1)
        elif res["n_survivors"]:
            r_max.append(primes[-1])
        else:
            r_max.append(max(r for r, c in zip(primes, cs) if c))
        if a % 10000 == 1:
            print("s6 p <= %d: %.0f s" % (b, time.time() - t), flush=True)
    out = dict(workload="s6", p0=1, p1=p_max, band_rows=band, primes=primes, counts=counts,
               n_pairs=pairs, n_survivors=surv, r_max=r_max, max_depth_prime=max(r_max),
               oracle_seconds=round(time.time() - t, 1))
    with open(os.path.join(HERE, "oracle_s6.json"), "w") as f:
        json.dump(out, f)
    print("s6 pairs", pairs, "survivors", surv, "depth", max(r_max), out["oracle_seconds"], "s")


if __name__ == "__main__":
    args = sys.argv[1:]
    threads = 0
    if "--threads" in args:
        k = args.index("--threads")
        threads = int(args[k + 1])
        del args[k:k + 2]
    names = args or ["c1", "c2", "c3", "c4s"]
    for nm in names:
        if nm == "c4s":
            c4_sample()
        elif nm == "c4":
            c4_full(threads)
        elif nm == "top":
            top_rows(threads or 6)
        elif nm == "s6":
            section6()
        else:
            square(nm)
