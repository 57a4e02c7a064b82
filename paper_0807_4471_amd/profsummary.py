"""Per-kernel, per-grid-size duration summary of a rocprofv3 database.

    python -m paper_0807_4471_amd.profsummary <run_results.db> [name-substring]

Groups dispatches by (kernel name, grid size, workgroup size) so launches of
one kernel template on different lattices are not averaged together.
"""
import sqlite3
import sys


def main(db, sub=""):
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


if __name__ == "__main__":
    main(*sys.argv[1:])
