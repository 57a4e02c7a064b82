"""Parity cases run against the NaN-poisoned-LDS debug build of the library
(started by test_gpu_lds_poison.py in a child process with SCLBM_LIBRARY
pointing at libsclbm_lds_poison.so).  Every kernel path that stages the
Psi/rho ring, on lattices with ragged strips and chunks, periodic and
walled, is run for a few steps and compared with the FP64 oracle: a ring
cell read without having been staged would be NaN and show up here.
Prints "ok <cases>" and exits 0 when every case matches."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
sys.path.insert(0, os.path.dirname(HERE))

import numpy as np  # noqa: E402

from helpers import WORKLOAD, oracle_run  # noqa: E402

STEPS = 6
# (nx, ny, boundary, tiling) -- tiling: (tile_x, tile_y, waves[, stacked])
CASES = [
    (70, 37, "periodic", (60, 8, 1)), (70, 37, "walls", (33, 5, 1)),
    (130, 41, "periodic", (124, 9, 2)), (130, 41, "walls", (100, 13, 2)),
    (300, 29, "periodic", (252, 7, 4)), (300, 29, "walls", (200, 30, 4)),
    (61, 23, "periodic", (60, 4, 4, 1)), (61, 23, "walls", (41, 4, 4, 1)),
    (97, 19, "periodic", (50, 8, 8, 1)), (97, 19, "walls", (57, 8, 8, 1)),
    (40, 3, "periodic", (40, 4, 1)), (40, 2, "walls", (40, 4, 4, 1)),
]


def check(m, ref, what, tol=1e-12):
    r, ux, uy = ref
    for a, b in ((m["rhoA"], r[0]), (m["rhoB"], r[1]), (m["ux"], ux), (m["uy"], uy)):
        if not np.isfinite(a).all():
            raise SystemExit(f"{what}: non-finite result (an unstaged ring cell was read)")
        if np.abs(a - b).max() > tol:
            raise SystemExit(f"{what}: differs from the oracle by {np.abs(a - b).max():.3g}")


def main():
    from paper_0807_4471_amd import sclbm
    assert sclbm.LIB_PATH.endswith("libsclbm_lds_poison.so"), sclbm.LIB_PATH
    n = 0
    for nx, ny, bnd, tl in CASES:
        kw = dict(WORKLOAD, wall_u=(0.0, 0.05)) if bnd == "walls" else dict(WORKLOAD)
        _, _, ref = oracle_run(nx, ny, STEPS, seed=3, boundary=bnd, **kw)
        for diag_every in (0, 1):   # plain steps, and steps with fused diagnostics
            s = sclbm.Simulation(nx, ny, storage="f64", boundary=bnd, diag_every=diag_every,
                                 **kw)
            s.set_tiling(*tl)
            s.init_random(3)
            s.step(STEPS)
            check(s.moments(), ref, f"{nx}x{ny} {bnd} {tl} diag_every={diag_every}")
            d = s.diagnostics()          # the diagnostics read-out pass
            if not np.isfinite(d["mass"]).all() or d["bad_sites"]:
                raise SystemExit(f"{nx}x{ny} {bnd}: diagnostics {d}")
            s.order_parameter()          # the order-parameter read-out pass
            n += 1
    # batches of mixed stacked tiles and sweep strips.  Step-wise mode only:
    # a persistent (cooperative) launch needs the device's global wave-sync
    # resource, which HIP grants one process at a time, and the parent test
    # process may hold it; both modes run the same per-item code.
    for mode in ("stepwise",):
        sims, refs, tls = [], [], []
        for nx, ny, bnd, tl in CASES:
            if tl[2] != 4:
                continue
            kw = dict(WORKLOAD, wall_u=(0.0, 0.05)) if bnd == "walls" else dict(WORKLOAD)
            s = sclbm.Simulation(nx, ny, storage="f64", boundary=bnd, **kw)
            s.init_random(3)
            sims.append(s)
            tls.append(tuple(tl) + (0,) * (5 - len(tl)))
            refs.append(oracle_run(nx, ny, STEPS, seed=3, boundary=bnd, **kw)[2])
        b = sclbm.Batch(sims, tls, mode=mode)
        b.step(STEPS)
        b.status()
        for s, r, tl in zip(sims, refs, tls):
            check(s.moments(), r, f"batch {mode} {s.nx}x{s.ny} {tl}")
            n += 1
    print(f"ok {n}", flush=True)


if __name__ == "__main__":
    main()
