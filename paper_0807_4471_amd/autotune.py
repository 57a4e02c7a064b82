"""Tile-shape autotuner for the fused step.

For a lattice (nx, ny), storage and boundary it enumerates the tilings the
library accepts -- stacked tiles (4 or 8 waves along y) and sweep strips
(1, 2 or 4 waves wide, chunk heights from 4 rows up, with or without the
store throttle) -- times each with HIP events on the caller's GPU, and keeps
the fastest (median of repeats; ties broken by candidate order, so the choice
is deterministic for a given table).  Results are cached in a JSON table per
GPU architecture (``tuning/<arch>.json`` next to this file), which
``tiling_for`` consults; sizes without an entry take the nearest tuned size
of the same storage and boundary, scaled to the lattice.

Batch tilings (``batch=True``) are restricted to what a batch launch
accepts: 4 waves, stacked tiles or sweep strips.  A batch is tuned as
a whole (``tune_batch``): each instance's own best tile (timed alone) is
one candidate policy; the others are "balanced" sweep strips whose chunk
heights give every tile about the same number of sites, sized so the
co-resident grid takes 1..8 tiles per step, with a floor on the chunk
height (short chunks re-read their 4 halo rows too often when a batch holds
few sites).  Policies are scored on several mixes at once (geometric mean
of each mix's time relative to its best policy), so the winner suits large
and small batches alike.  The winning policy (not the tiles of one
particular mix) is stored per storage type and applied to any mix by
``batch_plan``.  Every policy is tried in both execution modes (one
persistent launch per call, or one ordinary launch per step).

    python -m paper_0807_4471_amd.autotune --sizes 512 1024 4096 --storage f32
"""
from __future__ import annotations

import argparse
import json
import os
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE_DIR = os.path.join(HERE, "tuning")
ARCH = "gfx950"


def table_path(arch: str = ARCH) -> str:
    return os.path.join(TABLE_DIR, f"{arch}.json")


def load_table(arch: str = ARCH) -> dict:
    try:
        with open(table_path(arch)) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def save_table(table: dict, arch: str = ARCH):
    os.makedirs(TABLE_DIR, exist_ok=True)
    tmp = table_path(arch) + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    os.replace(tmp, table_path(arch))


# Storage types that share another's memory behaviour share its table rows.
TABLE_STORAGE = {"f16sr": "f16dev"}


def key(nx, ny, storage, boundary, batch=False) -> str:
    storage = TABLE_STORAGE.get(storage, storage)
    return f"{'batch/' if batch else ''}{storage}/{boundary}/{nx}x{ny}"


def _strip_width(nx: int, wmax: int) -> int:
    ns = -(-nx // wmax)
    return max(-(-nx // ns), min(32, nx))


def candidates(nx: int, ny: int, batch: bool = False) -> list:
    """Tilings (tile_x, tile_y, waves, stacked, throttle[, write_through]) in
    a fixed order."""
    out = []
    for rw in ((4,) if batch else (4, 8)):
        out.append((min(_strip_width(nx, 60), 60), rw, rw, 1, 0))
        if not batch:
            out.append((min(_strip_width(nx, 60), 60), rw, rw, 1, 0, 1))
    for cw in ((4,) if batch else (1, 2, 4)):
        W = _strip_width(nx, 64 * cw - 4)
        ns = -(-nx // W)
        heights = [h for h in (4, 8, 16, 32, 64, 128, 256) if h < ny] + [ny]
        # heights giving ~1, 2 and 3 resident workgroups of this width per CU
        for per_cu in (1, 2, 3):
            target = max(1, (256 * per_cu * 4 // cw) // ns) if not batch else 0
            if target:
                heights.append(max(4, -(-ny // target)))
        for H in sorted(set(min(max(h, 4), max(ny, 4)) for h in heights)):
            for th in (0, 1):
                out.append((W, H, cw, 0, th))
    seen, uniq = set(), []
    for c in out:
        if c not in seen:
            seen.add(c)
            uniq.append(c)
    return uniq


def measure(sim, tiling, steps: int, repeats: int = 3) -> float:
    """Median microseconds per step of `sim` with `tiling`."""
    import torch
    sim.set_tiling(*tiling)
    sim.step(max(2, steps // 10))
    times = []
    for _ in range(repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        sim.step(steps)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) * 1e3 / steps)
    return statistics.median(times)


def tune(nx: int, ny: int, storage: str = "f32", boundary: str = "periodic", batch=False,
         steps: int | None = None, table: dict | None = None, verbose=False, **phys) -> tuple:
    """Time every candidate and record the fastest in `table` (or the file)."""
    from . import sclbm
    own_table = table is None
    if own_table:
        table = load_table()
    sim = sclbm.Simulation(nx, ny, storage=storage, boundary=boundary,
                           wall_u=(0.0, 0.05) if boundary == "walls" else (0.0, 0.0), **phys)
    sim.init_random(1)
    if steps is None:  # about 20 ms of work per measurement at ~30 GLUPS
        steps = int(min(2000, max(10, 6e8 / (nx * ny))))
    results = []
    for c in candidates(nx, ny, batch):
        us = measure(sim, c, steps)
        results.append((us, c))
        if verbose:
            print(f"  {key(nx, ny, storage, boundary, batch)} {c}: {us:9.2f} us/step", flush=True)
    best_us, best = min(results, key=lambda r: r[0])
    table[key(nx, ny, storage, boundary, batch)] = {
        "tiling": list(best), "us_per_step": round(best_us, 3),
        "mlups": round(nx * ny / best_us, 1), "candidates": len(results)}
    if own_table:
        save_table(table)
    sim.close()
    return best


def tiling_for(nx: int, ny: int, storage: str = "f32", boundary: str = "periodic",
               batch: bool = False, table: dict | None = None):
    """Tuned tiling for this lattice, or one derived from the nearest tuned
    size (strip width recomputed, chunk height scaled); None if the table has
    nothing for this storage/boundary."""
    table = load_table() if table is None else table
    k = key(nx, ny, storage, boundary, batch)
    if k in table:
        return tuple(table[k]["tiling"])
    prefix = f"{'batch/' if batch else ''}{TABLE_STORAGE.get(storage, storage)}/{boundary}/"
    best = None
    for kk, v in table.items():
        if not kk.startswith(prefix):
            continue
        tx, ty = (int(a) for a in kk[len(prefix):].split("x"))
        d = abs((tx * ty) ** 0.5 - (nx * ny) ** 0.5)
        if best is None or d < best[0]:
            best = (d, tx, ty, v["tiling"])
    if best is None:
        return None
    _, tx, ty, t = best
    W, H, waves, stacked, throttle = t[:5]
    wt = t[5] if len(t) > 5 else 0
    if stacked:
        return (min(_strip_width(nx, 60), 60), H, waves, 1, throttle, wt)
    Wn = _strip_width(nx, 64 * waves - 4)
    Hn = max(4, min(ny, round(H * ny / ty)))
    return (Wn, Hn, waves, 0, throttle)


def policy_key(storage: str) -> str:
    return f"batch-policy/{TABLE_STORAGE.get(storage, storage)}"


def balanced_tilings(shapes, capacity: int, per_wg: int = 1, throttle: int = 0,
                     hmin: int = 4) -> list:
    """4-wave sweep strips (<= 252 columns) whose chunks hold about
    total_sites / (capacity * per_wg) sites each, and at least hmin rows."""
    shapes = list(shapes)
    total = sum(nx * ny for nx, ny in shapes)
    target = max(1.0, total / float(max(1, capacity * per_wg)))
    out = []
    for nx, ny in shapes:
        W = _strip_width(nx, 252)
        H = max(int(round(target / W)), hmin)
        H = max(min(4, ny), min(ny, H))
        out.append((W, H, 4, 0, throttle))
    return out


_capacity_cache = {}


def batch_capacity(sims, kind: int = 1) -> int:
    """Co-resident workgroups of the batch kernel of this storage and kind
    (0 stacked, 1 sweep, 2 both), from a throwaway plan."""
    from . import sclbm
    key_ = (sims[0].storage, kind)
    if key_ not in _capacity_cache:
        s = sims[0]
        if kind == 0:
            tl = [(min(_strip_width(s.nx, 60), 60), 4, 4, 1, 0)]
        else:
            tl = [(_strip_width(s.nx, 252), max(min(4, s.ny), min(s.ny, 16)), 4, 0, 0)]
        b = sclbm.Batch([s], tl)
        _capacity_cache[key_] = b.info()["capacity"]
        b.close()
    return _capacity_cache[key_]


def batch_plan(sims, table: dict | None = None, mode: str | None = None):
    """(tilings, mode) for a batch of Simulations (one storage type) under the
    tuned policy (the best one of `mode`, if given); without one, each
    instance's own batch entry (or default), persistent mode."""
    table = load_table() if table is None else table
    key = policy_key(sims[0].storage) + (f"/{mode}" if mode else "")
    pol = table.get(key) or {"policy": "table", "mode": mode or "persistent"}
    return policy_tilings(sims, pol, table), pol.get("mode", mode or "persistent")


def batch_tilings(sims, table: dict | None = None) -> list:
    """Tilings of `batch_plan`."""
    return batch_plan(sims, table)[0]


def _time_batch(sims, tilings, steps: int, repeats: int = 3, mode="persistent") -> float:
    """Median milliseconds of one batch step call of `steps` steps."""
    import torch
    from . import sclbm
    b = sclbm.Batch(sims, tilings, mode=mode)
    b.step(max(2, steps // 10))
    times = []
    for _ in range(repeats):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.step(steps)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    b.status()
    b.close()
    return statistics.median(times)


def batch_policies() -> list:
    """Candidate batch policies in a fixed order: execution mode x (each
    instance's own tile, or balanced sweep strips)."""
    out = []
    for mode in ("persistent", "stepwise"):
        out.append({"policy": "table", "mode": mode})
        for hmin in (8, 32):
            for per_wg in (1, 3, 6, 8):
                for th in (0, 1):
                    out.append({"policy": "balanced", "mode": mode, "per_wg": per_wg,
                                "throttle": th, "hmin": hmin})
    return out


def policy_tilings(sims, pol: dict, table: dict) -> list:
    from . import sclbm
    if pol["policy"] == "balanced":
        return balanced_tilings([(s.nx, s.ny) for s in sims], batch_capacity(sims, kind=1),
                                pol["per_wg"], pol["throttle"], pol.get("hmin", 4))
    out = []
    for s in sims:
        t = tiling_for(s.nx, s.ny, s.storage, s.boundary, batch=True, table=table)
        out.append(tuple(t) if t is not None else sclbm.default_batch_tiling(s.nx, s.ny))
    return out


def tune_batch(mixes, steps: int | None = None, table: dict | None = None,
               verbose=False) -> dict:
    """Time every candidate policy on each mix (a list of Simulation lists of
    one storage type); store the policy with the best geometric-mean time
    relative to each mix's fastest as that storage type's batch policy."""
    import math
    if mixes and not isinstance(mixes[0], (list, tuple)):
        mixes = [mixes]
    own_table = table is None
    if own_table:
        table = load_table()
    pols = batch_policies()
    times = []            # [mix][policy] us per step
    for sims in mixes:
        sites = sum(s.nx * s.ny for s in sims)
        n = steps if steps is not None else int(min(2000, max(10, 6e8 / sites)))
        row = []
        for pol in pols:
            ms = _time_batch(sims, policy_tilings(sims, pol, table), n,
                             mode=pol.get("mode", "persistent"))
            row.append(ms / n * 1e3)
            if verbose:
                print(f"  [{len(sims)} inst, {sites} sites] {pol}: {row[-1]:9.2f} us/step  "
                      f"{sites / row[-1]:9.1f} MLUPS", flush=True)
        times.append(row)
    score = [math.exp(sum(math.log(times[m][p] / min(times[m])) for m in range(len(mixes)))
                      / len(mixes)) for p in range(len(pols))]
    def record(best):
        rec = dict(pols[best])
        rec.update({"score": round(score[best], 4), "candidates": len(pols),
                    "mixes": [{"instances": len(sims), "sites": sum(s.nx * s.ny for s in sims),
                               "us_per_step": round(times[m][best], 3),
                               "best_us_per_step": round(min(times[m]), 3)}
                              for m, sims in enumerate(mixes)]})
        return rec
    key = policy_key(mixes[0][0].storage)
    for mode in ("persistent", "stepwise"):   # best of each mode, for callers that need one
        idx = [p for p in range(len(pols)) if pols[p].get("mode", "persistent") == mode]
        table[f"{key}/{mode}"] = record(min(idx, key=lambda p: score[p]))
    rec = record(min(range(len(pols)), key=lambda p: score[p]))
    table[key] = rec
    if own_table:
        save_table(table)
    return rec


def policy_mixes(storage: str) -> list:
    """The three mixes a batch policy is scored on: the 64-instance uneven
    batch workload, a serving-like group of 8 lattices (64^2..1024^2, half
    of them between walls) and one 1024^2 lattice; every instance
    initialised from its seed."""
    from . import sclbm
    from .inputs import batch_mix
    W = dict(Ga=(-12.55, -11.80), Gr=(11.70, 10.95), Gx=0.58, rho0=0.70)

    def sim(nx, ny, seed, boundary="periodic", **kw):
        s = sclbm.Simulation(nx, ny, storage=storage, boundary=boundary,
                             wall_u=(0.0, 0.05) if boundary == "walls" else (0.0, 0.0),
                             **{**W, **kw})
        return s.init_random(seed)

    mix64 = [sim(m["nx"], m["ny"], m["seed"], rho0=m["rho0"], Gx=m["Gx"], tau=m["tau"])
             for m in batch_mix()]
    serving_like = [sim(n, n, 10 + k, "walls" if k % 2 else "periodic")
                    for k, n in enumerate((64, 96, 150, 230, 350, 520, 700, 1024))]
    return [mix64, serving_like, [sim(1024, 1024, 7)]]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", type=int, nargs="+", default=[64, 128, 256, 512, 1024, 2048, 4096])
    ap.add_argument("--shapes", nargs="+", default=[],
                    help="rectangular lattices NXxNY to tune instead of the square sizes "
                         "(e.g. 8192x1024, one GPU's slab of a lattice split by rows)")
    ap.add_argument("--storage", nargs="+", default=["f32", "f16dev", "f64"])
    ap.add_argument("--boundary", nargs="+", default=["periodic"])
    ap.add_argument("--batch", action="store_true")
    ap.add_argument("--policy", action="store_true",
                    help="tune the batch policy (tile policy x execution mode) of each storage "
                         "on the three mixes of policy_mixes, instead of single lattices")
    ap.add_argument("--verbose", action="store_true")
    a = ap.parse_args()
    table = load_table()
    if a.policy:
        for st in a.storage:
            mixes = policy_mixes(st)
            rec = tune_batch(mixes, table=table, verbose=a.verbose)
            print(f"{policy_key(st)}: {rec}", flush=True)
            save_table(table)
            for m in mixes:
                for s in m:
                    s.close()
        return
    if a.shapes:
        shapes = [tuple(int(v) for v in sh.lower().split("x")) for sh in a.shapes]
    else:
        shapes = [(n, n) for n in a.sizes]
    for st in a.storage:
        for bc in a.boundary:
            for nx, ny in shapes:
                best = tune(nx, ny, st, bc, batch=a.batch, table=table, verbose=a.verbose)
                e = table[key(nx, ny, st, bc, a.batch)]
                print(f"{key(nx, ny, st, bc, a.batch)}: {best}  {e['us_per_step']} us/step  "
                      f"{e['mlups']} MLUPS", flush=True)
                save_table(table)


if __name__ == "__main__":
    main()
