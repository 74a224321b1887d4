"""Writes the oracle's expected values for the rectangle workloads into
tests/golden/oracle_<name>.json.  Calls only the oracle package.

Workloads (sieve over all coprime p != q in the square, primes as listed):
  c1  1 <= p, q <= 200,    primes 3..31
  c2  1 <= p, q <= 10^4,   primes 3..97
  c3  1 <= p, q <= 10^5,   primes 3..997
  c4s a seeded sample of the batched workload's rectangles, primes 3..499
  s6  region (1.2) for p = 1..154000, primes 11..541 (the scan of section 6),
      per hundred of p: the deepest prime some pair was tested against

usage: python tests/golden/make_golden.py [c1 c2 c3 c4s s6]
"""
import json
import os
import sys
import time

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
    names = sys.argv[1:] or ["c1", "c2", "c3", "c4s"]
    for nm in names:
        if nm == "c4s":
            c4_sample()
        elif nm == "s6":
            section6()
        else:
            square(nm)
