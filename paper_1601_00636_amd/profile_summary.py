"""Summaries of rocprofv3 result databases (SQLite, rocpd schema) as markdown.

usage:
  python -m paper_1601_00636_amd.profile_summary trace DB "COMMAND"
  python -m paper_1601_00636_amd.profile_summary traffic FETCH_DB WRITE_DB COPY_FETCH_DB COPY_WRITE_DB "COMMANDS"
  python -m paper_1601_00636_amd.profile_summary counters DB1,DB2 "COMMANDS" UNITS

`trace`: per-kernel dispatch counts and durations of a --kernel-trace run.
`counters`: SQ counters of the sweep's largest dispatches per launch and per
64x64 unit (profiles/sweep_counters.json, one record per kernel instance,
keyed by the source hash as below).
`traffic`: FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the sweep kernel's
largest launches, scaled by what the same counters read for a device copy of
2^30 bytes (bench.py --calibrate-copy), and writes profiles/sweep_traffic.json
keyed by the SHA-256 of the sweep kernel's source so that bench.py stops
reporting the figure once that source changes.
"""
import hashlib
import json
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SWEEP_SRC = os.path.join(HERE, "csrc", "kernels_sieve.hip")
COPY_BYTES = 1 << 30


def sweep_source_hash():
    with open(SWEEP_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _short(name):
    name = name.replace("(anonymous namespace)::", "").replace("cuboid::", "")
    return name.split("(")[0][:80]


def trace(db, command):
    c = sqlite3.connect(db)
    rows = list(c.execute(
        "select name, count(*), sum(duration), avg(duration), min(duration), max(duration) "
        "from kernels group by name order by sum(duration) desc limit 20"))
    total = sum(r[2] for r in rows) or 1
    out = ["# rocprofv3 kernel trace\n\n", "Command:\n\n    %s\n\n" % command,
           "| kernel | calls | total ms | avg us | min us | max us | % |\n",
           "|---|---|---|---|---|---|---|\n"]
    for n, k, tot, avg, mn, mx in rows:
        out.append("| %s | %d | %.3f | %.1f | %.1f | %.1f | %.1f |\n"
                   % (_short(n), k, tot / 1e6, avg / 1e3, mn / 1e3, mx / 1e3, 100.0 * tot / total))
    out.append("\nLargest sweep launches (grid in work-items, LDS bytes, duration):\n\n")
    out.append("| kernel | grid | LDS | us |\n|---|---|---|---|\n")
    for n, g, l, d in c.execute("select name, grid_x, lds_size, duration from kernels where name "
                                "like '%sweep%' order by duration desc limit 8"):
        out.append("| %s | %d | %d | %.1f |\n" % (_short(n), g, l, d / 1e3))
    return "".join(out)


def _counter(db, counter, like):
    c = sqlite3.connect(db)
    return list(c.execute("select kernel_name, value, duration from counters_collection where "
                          "counter_name=? and kernel_name like ? order by duration desc",
                          (counter, like)))


def traffic(fetch_db, write_db, cfetch_db, cwrite_db, command, launches=4):
    f = _counter(fetch_db, "FETCH_SIZE", "%sweep%")[:launches]
    w = _counter(write_db, "WRITE_SIZE", "%sweep%")[:launches]
    cf = _counter(cfetch_db, "FETCH_SIZE", "%copyBuffer%")
    cw = _counter(cwrite_db, "WRITE_SIZE", "%copyBuffer%")
    cf_kib = sum(x[1] for x in cf) / len(cf)
    cw_kib = sum(x[1] for x in cw) / len(cw)
    fscale = COPY_BYTES / (cf_kib * 1024)
    wscale = COPY_BYTES / (cw_kib * 1024)
    fk = sum(x[1] for x in f) / len(f)
    wk = sum(x[1] for x in w) / len(w)
    dur_ns = sum(x[2] for x in f) / len(f)
    traffic_b = fk * 1024 * fscale + wk * 1024 * wscale
    rec = {"kernel_source_sha256": sweep_source_hash(), "kernel": _short(f[0][0]),
           "fetch_kib_per_launch": fk, "write_kib_per_launch": wk,
           "copy_fetch_kib": cf_kib, "copy_write_kib": cw_kib,
           "fetch_scale": fscale, "write_scale": wscale,
           "traffic_bytes_per_launch": traffic_b, "launch_ns": dur_ns,
           "traffic_GBps": traffic_b / dur_ns}
    md = ["# HBM traffic of the sweep kernel (batched 4096-rectangle workload)\n\n",
          "Commands (one counter per run):\n\n    %s\n\n" % command.replace(";", "\n   "),
          "| quantity | value |\n|---|---|\n",
          "| kernel | %s |\n" % rec["kernel"],
          "| FETCH_SIZE per launch (KiB, mean of %d largest) | %.1f |\n" % (len(f), fk),
          "| WRITE_SIZE per launch (KiB) | %.1f |\n" % wk,
          "| copy of 2^30 B: FETCH_SIZE (KiB) | %.1f |\n" % cf_kib,
          "| copy of 2^30 B: WRITE_SIZE (KiB) | %.1f |\n" % cw_kib,
          "| fetch scale (bytes per counted byte) | %.4f |\n" % fscale,
          "| write scale | %.4f |\n" % wscale,
          "| HBM bytes per launch (scaled) | %.4g |\n" % traffic_b,
          "| launch duration (ms) | %.3f |\n" % (dur_ns / 1e6),
          "| HBM rate (GB/s) | %.1f |\n" % rec["traffic_GBps"],
          "| sweep source sha256 | %s |\n" % rec["kernel_source_sha256"]]
    return "".join(md), rec


def counters(dbs, command, units):
    """SQ counters of the largest sweep dispatches, per dispatch and per unit;
    also writes profiles/sweep_counters.json keyed by the sweep source's hash
    (bench.py turns the per-unit figures into issue fractions while the
    source is unchanged)."""
    rows = {}
    kernel = None
    for db in dbs:
        c = sqlite3.connect(db)
        for kname, name, v, d in c.execute(
                "select kernel_name, counter_name, value, duration from counters_collection where "
                "kernel_name like '%sweep%' order by duration desc"):
            rows.setdefault(name, []).append((d, v))
            kernel = kernel or _short(kname)
    rec = {"kernel_source_sha256": sweep_source_hash(), "kernel": kernel,
           "units_per_launch": units, "per_unit": {}}
    for name in sorted(rows):
        top = sorted(rows[name], reverse=True)[:2]
        rec["per_unit"][name] = sum(x[1] for x in top) / len(top) / units
    _merge_record(os.path.join(ROOT, "profiles", "sweep_counters.json"), rec)
    out = ["# SQ counters of the sweep kernel (batched 4096-rectangle workload)\n\n",
           "Commands (one counter group per run):\n\n    %s\n\n" % command.replace(";", "\n   "),
           "Averages over the 2 largest dispatches (the timed batched launches); "
           "%d 64x64 units per launch.\n\n" % units,
           "| counter | per dispatch | per unit |\n|---|---|---|\n"]
    for name in sorted(rows):
        top = sorted(rows[name], reverse=True)[:2]
        v = sum(x[1] for x in top) / len(top)
        out.append("| %s | %.4g | %.2f |\n" % (name, v, v / units))
    return "".join(out)


def _merge_record(path, rec):
    """Keep one record per sweep kernel instance in a profiles JSON file
    ({"records": [...]}), replacing an older record of the same instance."""
    recs = []
    try:
        with open(path) as f:
            old = json.load(f)
        recs = old.get("records", [old] if "kernel_source_sha256" in old else [])
    except (OSError, ValueError):
        pass
    recs = [r for r in recs if r.get("kernel") != rec["kernel"]] + [rec]
    with open(path, "w") as f:
        json.dump({"records": recs}, f, indent=1)


def main(argv):
    if argv[0] == "trace":
        print(trace(argv[1], argv[2]))
    elif argv[0] == "counters":
        print(counters(argv[1].split(","), argv[2], int(argv[3])))
    elif argv[0] == "traffic":
        md, rec = traffic(argv[1], argv[2], argv[3], argv[4], argv[5])
        print(md)
        _merge_record(os.path.join(ROOT, "profiles", "sweep_traffic.json"), rec)
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
