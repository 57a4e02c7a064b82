"""Summaries of rocprofv3 output for the step kernels.

    python -m paper_0807_4471_amd.profsummary db <run_results.db> [name-substring]
    python -m paper_0807_4471_amd.profsummary stats <kernel_stats.csv> [name-substring]
    python -m paper_0807_4471_amd.profsummary trace <kernel_trace.csv> [name-substring]
    python -m paper_0807_4471_amd.profsummary traffic \\
        --fetch <FETCH_SIZE counter_collection.csv> --write <WRITE_SIZE ...csv> \\
        --copy-fetch <csv> --copy-write <csv> --copy-bytes 1073741824 \\
        --entry KEY=NAME_SUBSTRING@GRID [...] -o traffic_counters.json

`db` groups the dispatches of a rocpd database by (kernel name, grid size,
workgroup size), so launches of one kernel template on different lattices
are not averaged together; `trace` does the same for a kernel_trace.csv.
`stats` prints a kernel_stats.csv in microseconds.

`traffic` turns two counter runs (FETCH_SIZE, then WRITE_SIZE: KiB moved
between L2 and the memory fabric per dispatch) into bytes per launch of the
kernels named by the --entry options.  Each counter is scaled by what it
reads for a plain device copy of --copy-bytes bytes (the largest dispatch in
the copy runs), so the figures are in true bytes whatever the counter's own
unit.  The output records the hash of the kernel source the counters were
taken on; readers treat the figures as stale once the source changes.
"""
from __future__ import annotations

import argparse
import csv
import json
import sqlite3
import sys
from collections import defaultdict


def cmd_db(db, sub=""):
    c = sqlite3.connect(db)
    q = ("select name, grid_x, workgroup_x, count(*), avg(duration), min(duration), "
         "max(duration), vgpr_count, accum_vgpr_count, sgpr_count, lds_size "
         "from kernels group by name, grid_x, workgroup_x order by sum(duration) desc")
    print(f"{'kernel':70s} {'grid':>8s} {'wg':>4s} {'calls':>6s} {'avg_us':>9s} "
          f"{'min_us':>9s} {'max_us':>9s} vgpr agpr sgpr lds")
    for name, gx, wx, n, avg, mn, mx, v, a, s, lds in c.execute(q):
        if sub and sub not in name:
            continue
        short = name.replace("sclbm::", "").split("(")[0][:70]
        print(f"{short:70s} {gx:8d} {wx:4d} {n:6d} {avg / 1e3:9.3f} {mn / 1e3:9.3f} "
              f"{mx / 1e3:9.3f} {v:4d} {a:4d} {s:4d} {lds}")


def cmd_stats(path, sub=""):
    print(f"| kernel | calls | avg us | min us | max us | share % |")
    print(f"|---|---:|---:|---:|---:|---:|")
    for r in csv.DictReader(open(path)):
        if sub and sub not in r["Name"]:
            continue
        short = r["Name"].replace("sclbm::", "").split("(")[0]
        print(f"| `{short}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.3f} | "
              f"{float(r['MinNs']) / 1e3:.3f} | {float(r['MaxNs']) / 1e3:.3f} | "
              f"{float(r['Percentage']):.2f} |")


def cmd_trace(path, sub=""):
    groups = defaultdict(list)
    for r in csv.DictReader(open(path)):
        if sub and sub not in r["Kernel_Name"]:
            continue
        dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        g = int(r.get("Grid_Size_X") or r["Grid_Size"])
        w = int(r.get("Workgroup_Size_X") or r["Workgroup_Size"])
        groups[(r["Kernel_Name"], g, w)].append(dur)
    print("| kernel | grid | workgroup | calls | avg us | median us | min us | max us |")
    print("|---|---:|---:|---:|---:|---:|---:|---:|")
    for (name, g, w), d in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        d = sorted(d)
        short = name.replace("sclbm::", "").split("(")[0]
        print(f"| `{short}` | {g} | {w} | {len(d)} | {sum(d) / len(d):.3f} | "
              f"{d[len(d) // 2]:.3f} | {d[0]:.3f} | {d[-1]:.3f} |")


def _per_dispatch(path):
    """{(kernel name, grid size): [counter value per dispatch]}"""
    out = defaultdict(list)
    for r in csv.DictReader(open(path)):
        out[(r["Kernel_Name"], int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
    return out


def _copy_factor(path, nbytes):
    vals = [v for vs in _per_dispatch(path).values() for v in vs]
    top = max(vals)
    return nbytes / (top * 1024.0), top


def _match(table, spec):
    sub, grid = spec.rsplit("@", 1)
    hits = [(k, v) for k, v in table.items() if sub in k[0] and k[1] == int(grid)]
    if len(hits) != 1:
        raise SystemExit(f"entry {spec!r} matches {len(hits)} kernels")
    return hits[0]


def cmd_traffic(argv):
    ap = argparse.ArgumentParser(prog="profsummary traffic")
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--copy-bytes", type=int, required=True)
    ap.add_argument("--entry", action="append", required=True, help="KEY=NAME_SUBSTRING@GRID")
    ap.add_argument("-o", "--out", required=True)
    a = ap.parse_args(argv)
    from .build import kernel_source_hash
    ff, fraw = _copy_factor(a.copy_fetch, a.copy_bytes)
    fw, wraw = _copy_factor(a.copy_write, a.copy_bytes)
    fetch, write = _per_dispatch(a.fetch), _per_dispatch(a.write)
    res = {"kernel_hash": kernel_source_hash(),
           "calibration": {"copy_bytes": a.copy_bytes, "copy_fetch_kib": fraw,
                           "copy_write_kib": wraw, "fetch_factor": ff, "write_factor": fw},
           "per_launch_bytes": {}, "detail": {}}
    for e in a.entry:
        key, spec = e.split("=", 1)
        (name, grid), fv = _match(fetch, spec)
        (_, _), wv = _match(write, spec)
        fb = sum(fv) / len(fv) * 1024.0 * ff
        wb = sum(wv) / len(wv) * 1024.0 * fw
        res["per_launch_bytes"][key] = round(fb + wb)
        res["detail"][key] = {"kernel": name.split("(")[0], "grid": grid,
                              "dispatches": [len(fv), len(wv)],
                              "fetch_bytes": round(fb), "write_bytes": round(wb)}
    with open(a.out, "w") as fh:
        json.dump(res, fh, indent=1, sort_keys=True)
        fh.write("\n")
    print(json.dumps(res, indent=1, sort_keys=True))


def main(argv):
    if not argv:
        raise SystemExit(__doc__)
    cmd, rest = argv[0], argv[1:]
    if cmd == "db":
        cmd_db(*rest)
    elif cmd == "stats":
        cmd_stats(*rest)
    elif cmd == "trace":
        cmd_trace(*rest)
    elif cmd == "traffic":
        cmd_traffic(rest)
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
