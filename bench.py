#!/usr/bin/env python3
"""Throughput benchmark of the fused two-species Shan-Chen LBM step on one
MI355X.

Headline workload: the micro-emulsion lattice, 512x512 periodic, FP32
populations, caption couplings (G_A1=-12.55, G_A2=11.70, G_B1=-11.80,
G_B2=10.95, G^X=0.58), rho0 = 0.70, Psi = rho0 (1 - exp(-rho/rho0)),
tau_A = tau_B = 1, densities 0.7 (1 + 0.05 U) from seed 1, fused FP64
diagnostics every 1000 steps.  One step = one fused stream + force +
collide pass over the lattice (plus the diagnostics reduction on every
1000th step).  Inputs are resident in HBM before timing starts.

Prints ONE JSON line (see the keys below).  `value` is two-species MLUPS
(1 LUP = one site advanced one step, both species).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
BYTES_PER_LUP = {"f64": 288, "f32": 144, "f16dev": 72}
WORKLOAD = dict(Ga=(-12.55, -11.80), Gr=(11.70, 10.95), Gx=0.58, rho0=0.70)
KERNEL_SOURCES = ["paper_0807_4471_amd/csrc/sclbm_kernels.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--nx", type=int, default=512)
    ap.add_argument("--storage", default="f32", choices=list(BYTES_PER_LUP))
    ap.add_argument("--rho0", type=float, default=0.70)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dram", action="store_true", help="skip the DRAM-resident side runs")
    ap.add_argument("--cpu-steps", type=int, default=80)
    return ap.parse_args()


def run_gpu(nx, storage, steps, warmup, rho0, diag_every, torch, sclbm):
    kw = dict(WORKLOAD, rho0=rho0)
    sim = sclbm.Simulation(nx, nx, storage=storage, diag_every=diag_every,
                           rho_ref=(0.7, 0.7), **kw)
    sim.init_random(1, mean=(0.7, 0.7), amp=0.05)
    d0 = sim.diagnostics()
    sim.step(warmup)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(st)
    sim.step(steps)
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    d = sim.diagnostics()
    d["mass0"] = d0["mass"]
    return sim, ms_total, wall, d


def roofline(nx, storage, kernel_ms):
    """Roofline of the fused step kernel.  kernel_ms is its average launch
    duration: the HIP-event time of the timed region on the launch stream
    divided by the number of step launches (the launches run back to back;
    the few diagnostics reductions inside the region add < 0.1%)."""
    alg = BYTES_PER_LUP[storage] * nx * nx
    achieved = alg / (kernel_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
            "alg_bytes_per_launch": alg, "kernel_us": round(kernel_ms * 1e3, 3)}


def traffic_for(key: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t.get("per_launch_bytes", {}).get(key)


def cpu_baseline(nx, steps, rho0):
    import numpy as np
    import oracle
    from paper_0807_4471_amd import inputs
    oracle.build(force=False)
    p = oracle.Params(nx=nx, ny=nx, **dict(WORKLOAD, rho0=rho0))
    f = oracle.init(p, inputs.random_densities(nx, nx, 1))
    t0 = time.perf_counter()
    oracle.run(p, f, steps)
    dt = time.perf_counter() - t0
    assert np.isfinite(f).all()
    return {"value": round(nx * nx * steps / dt / 1e6, 4), "unit": "MLUPS", "cores": 1,
            "kind": "oracle",
            "sample": f"FP64 oracle, {nx}x{nx} periodic, same couplings and seeded init, "
                      f"{steps} steps ({dt:.1f} s, single thread)"}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {a.gpus} is not supported "
              "(the lattice would shard into y-slabs with halo exchange; not built).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_0807_4471_amd import sclbm
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(3)
    nx, storage = a.nx, a.storage
    sim, ms_total, wall, d = run_gpu(nx, storage, a.steps, a.warmup, a.rho0, 1000, torch, sclbm)
    ms_step = ms_total / a.steps
    mlups = nx * nx / (ms_step * 1e-3) / 1e6
    roof = roofline(nx, storage, ms_step)
    roof["traffic"] = traffic_for(f"{storage}_{nx}")
    # ping-pong footprint (2 copies x 18 populations) vs the 256 MiB Infinity Cache
    roof["cache_resident"] = BYTES_PER_LUP[storage] * nx * nx < 256 * 2 ** 20
    out = {
        "metric": "two-species MLUPS and % HBM roofline; p50/p99 latency of served solves",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "f16dev": "f32 (f16 storage)"}[storage],
        "data": "synthetic",
        "config": {"workload": f"micro-emulsion {nx}x{nx} periodic two-species D2Q9 "
                               f"Shan-Chen, {storage} populations, rho0={a.rho0}, "
                               "A=rho0, caption couplings, tau=1, 5% random init",
                   "nx": nx, "ny": nx, "storage": storage, "diag_every": 1000,
                   "tiling": list(sim.get_tiling())},
        "roofline": roof,
        "mass_drift": [float(abs(d["mass"][s] / d["mass0"][s] - 1.0)) for s in (0, 1)],
        "wall_s": round(wall, 3),
    }
    del sim
    if not a.no_dram:
        side = []
        for st_, n_ in (("f32", 4096), ("f16dev", 4096), ("f64", 2048)):
            s2, mt, _, _ = run_gpu(n_, st_, 200, 20, a.rho0, 0, torch, sclbm)
            r = roofline(n_, st_, mt / 200)
            r["traffic"] = traffic_for(f"{st_}_{n_}")
            side.append({"workload": f"{n_}x{n_} {st_} (DRAM-resident)",
                         "mlups": round(n_ * n_ / (mt / 200 * 1e-3) / 1e6, 1), "roofline": r,
                         "tiling": list(s2.get_tiling())})
            del s2
            torch.cuda.empty_cache()
        out["dram_resident"] = side
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(nx, a.cpu_steps, a.rho0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
