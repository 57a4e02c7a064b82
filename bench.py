#!/usr/bin/env python3
"""Throughput benchmark of the fused two-species Shan-Chen LBM step on one
MI355X.

Headline workload (`value`): the micro-emulsion lattice, 512x512 periodic,
FP32 populations, caption couplings (G_A1=-12.55, G_A2=11.70, G_B1=-11.80,
G_B2=10.95, G^X=0.58), rho0 = 0.70, Psi = rho0 (1 - exp(-rho/rho0)),
tau_A = tau_B = 1, densities 0.7 (1 + 0.05 U) from seed 1, fused FP64
diagnostics every 1000 steps, tile shape from the tuned table.  One step =
one fused stream + force + collide pass over the lattice (plus the
diagnostics reduction on every 1000th step).  Inputs are resident in HBM
before timing starts; the timed region is bracketed by device syncs and
timed with HIP events on the launch stream, its launches queued behind a
short GPU-side sleep so that host launch latency is not measured.

Side objects in the same JSON line:
  rho0_sweep     FP32 at rho0 in {0.60, 0.70, 0.75}, same steps, against the
                 FP64 GPU path (mass drift, structure-factor peak)
  dram_resident  lattices larger than the 256 MiB Infinity Cache
  sheared_cell   1024x1024 between walls (top at U = 0.01, 0.05, 0.1):
                 mean shear stress and apparent viscosity, FP32 and FP16
                 storage against the FP64 path
  rheology       128x128 under the Kolmogorov force: response R(t) and
                 interface indicator I_AB(t)
  ageing         overlap C(t_w, tau) of the order parameter over an ensemble
                 of such lattices advanced as one batch
  laplace        nominal surface tension sigma(rho0) from batched static
                 droplets, both Psi amplitudes
  batch          64 uneven instances in one persistent launch per call,
                 against the same instances stepped one launch at a time
  serving        a Poisson trace served with continuous batching, against
                 the same trace served one request at a time on the FP64 path
  roofline       of the step kernel of the headline workload
  cpu_baseline   the FP64 oracle on the host, on a bounded sample

Prints ONE JSON line.  `value` is two-species MLUPS (1 LUP = one site
advanced one step, both species).

    python bench.py                      # everything, N = 1
    python bench.py --calibrate-copy     # plain copy for the counter scale
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
BYTES_PER_LUP = {"f64": 288, "f32": 144, "f16dev": 72, "f16sr": 72}
WORKLOAD = dict(Ga=(-12.55, -11.80), Gr=(11.70, 10.95), Gx=0.58, rho0=0.70)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")
METRIC = "two-species MLUPS and % HBM roofline; p50/p99 latency of served solves"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    from paper_0807_4471_amd.build import kernel_source_hash
    return kernel_source_hash()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--nx", type=int, default=512)
    ap.add_argument("--storage", default="f32", choices=list(BYTES_PER_LUP))
    ap.add_argument("--rho0", type=float, default=0.70)
    ap.add_argument("--forcing", default="shift", choices=["shift", "guo"],
                    help="force coupling of the headline run")
    ap.add_argument("--no-guo", action="store_true",
                    help="skip the Guo-forcing side run of the headline workload")
    ap.add_argument("--no-sweep", action="store_true", help="skip the rho0 sweep")
    ap.add_argument("--no-dram", action="store_true", help="skip the DRAM-resident side runs")
    ap.add_argument("--no-small", action="store_true", help="skip the 64x64 FP64 case")
    ap.add_argument("--no-shear", action="store_true", help="skip the sheared-cell object")
    ap.add_argument("--shear-steps", type=int, default=50000)
    ap.add_argument("--shear-seeds", type=int, default=4,
                    help="FP64 seeds of the sheared cell (run-to-run spread)")
    ap.add_argument("--no-rheology", action="store_true", help="skip the Kolmogorov-flow run")
    ap.add_argument("--rheology-steps", type=int, default=500000)
    ap.add_argument("--rheology-storage", default="f32", choices=list(BYTES_PER_LUP))
    ap.add_argument("--no-ageing", action="store_true", help="skip the ageing ensemble")
    ap.add_argument("--ageing-members", type=int, default=16)
    ap.add_argument("--no-laplace", action="store_true", help="skip the sigma(rho0) sweep")
    ap.add_argument("--laplace-steps", type=int, default=10000)
    ap.add_argument("--laplace-forcing", default="shift", choices=["shift", "guo"],
                    help="force coupling of the droplets of the sigma(rho0) sweep")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=20000)
    ap.add_argument("--batch-modes", default="stepwise,persistent",
                    help="batch execution modes to time (a profiler run leaves out "
                         "'persistent', whose cooperative launch rocprofv3 does not survive "
                         "at exit)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=100)
    ap.add_argument("--serve-load", type=float, default=0.8)
    ap.add_argument("--serve-legs", default="step,work,seq",
                    help="services to run on the trace: step (batched, step-fair), "
                         "work (batched, work-fair), seq (one at a time, FP64)")
    ap.add_argument("--serve-capacity-glups", type=float, default=None,
                    help="batch capacity that sets the arrival rate (default: the "
                         "measured batch rate, else 20)")
    ap.add_argument("--device-warmup-ms", type=float, default=DEVICE_WARMUP_MS,
                    help="before each single-lattice timed region, run the step kernel on a "
                         "scratch lattice of the same shape for this long (0: off)")
    ap.add_argument("--repeats", type=int, default=5,
                    help="further 20k-step timed regions of the headline lattice, for the "
                         "run-to-run spread (0: none, e.g. under a profiler)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-scale", type=float, default=1.0,
                    help="scale of the oracle timing sample's step counts")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (counter calibration)")
    return ap.parse_args()


def timed(torch, fn):
    """HIP-event milliseconds of fn() on the current stream, plus wall s.

    The launches fn() enqueues are queued behind a short GPU-side sleep
    (2e5 clock cycles, before the start event), so the region starts with
    its work already queued: the host's launch latency, which a short region
    (e.g. 20 steps) would otherwise pay before and between its first
    kernels, is not in the measured GPU time.  The region still times
    exactly the work fn() enqueues."""
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if hasattr(torch.cuda, "_sleep"):
        torch.cuda._sleep(200_000)
    e0.record(st)
    fn()
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1), time.perf_counter() - t0


DEVICE_WARMUP_MS = 20.0


def device_warmup(nx, ny, storage, rho0, forcing, torch, sclbm, ms=None):
    """Bring the device to its steady state for this kernel before a timed
    region: the same step kernel on a scratch lattice of the same shape and
    storage (its own state; the timed lattice gets exactly its warm-up
    steps) for `ms` milliseconds.  Measured: after a 5-step warm-up the
    first 20-step region of the 512^2 lattice runs at 9.3 us per step, at
    8.8-9.0 after this; a device copy or matrix products of the same
    duration do not do it."""
    ms = DEVICE_WARMUP_MS if ms is None else ms
    if ms <= 0:
        return
    w = sclbm.Simulation(nx, ny, storage=storage, rho_ref=(0.7, 0.7), tiling="auto",
                         **dict(WORKLOAD, rho0=rho0, forcing=forcing))
    w.init_random(2, mean=(0.7, 0.7), amp=0.05)
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < ms:
        w.step(64)
        torch.cuda.synchronize()
    w.close()


def run_gpu(nx, storage, steps, warmup, rho0, diag_every, torch, sclbm, tiling="auto",
            forcing="shift", ny=None):
    kw = dict(WORKLOAD, rho0=rho0, forcing=forcing)
    ny = nx if ny is None else ny
    sim = sclbm.Simulation(nx, ny, storage=storage, diag_every=diag_every,
                           rho_ref=(0.7, 0.7), tiling=tiling, **kw)
    sim.init_random(1, mean=(0.7, 0.7), amp=0.05)
    d0 = sim.diagnostics()
    sim.step(warmup)
    device_warmup(nx, ny, storage, rho0, forcing, torch, sclbm)
    ms_total, wall = timed(torch, lambda: sim.step(steps))
    d = sim.diagnostics()
    d["mass0"] = d0["mass"]
    return sim, ms_total, wall, d


def roofline(nx, storage, kernel_ms, ny=None):
    """Roofline of the fused step kernel.  kernel_ms is its average launch
    duration: the HIP-event time of the timed region on the launch stream
    divided by the number of step launches (the launches run back to back;
    the diagnostics reductions inside the region add < 0.1%).  Algorithmic
    bytes: every site reads and writes 18 populations once."""
    alg = BYTES_PER_LUP[storage] * nx * (nx if ny is None else ny)
    achieved = alg / (kernel_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
            "alg_bytes_per_launch": alg, "kernel_us": round(kernel_ms * 1e3, 3)}


def with_traffic(r: dict, traffic):
    """Attach the counter bytes per launch and the rate they imply."""
    r["traffic"] = traffic
    if traffic:
        r["traffic_GBps"] = round(traffic / (r["kernel_us"] * 1e-6) / 1e9, 1)
    return r


def traffic_for(key: str):
    """Bytes per launch between L2 and the memory fabric, from committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs scaled by a plain copy, if they
    were taken on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t.get("per_launch_bytes", {}).get(key)


def structure_peak(torch, sim):
    """Peak (|k| shell, S) of the radially averaged structure factor of
    phi = rho_A - rho_B (k in units of 2 pi / L)."""
    import numpy as np
    m = sim.moments()
    phi = m["rhoA"] - m["rhoB"]
    ny, nx = phi.shape
    F = np.fft.fft2(phi - phi.mean())
    S = (np.abs(F) ** 2) / (nx * ny)
    K = np.sqrt((np.fft.fftfreq(ny) * ny)[:, None] ** 2 + (np.fft.fftfreq(nx) * nx)[None, :] ** 2)
    shell = np.rint(K).astype(int)
    tot = np.bincount(shell.ravel(), S.ravel())
    cnt = np.bincount(shell.ravel())
    Sk = np.where(cnt > 0, tot / np.maximum(cnt, 1), 0.0)
    Sk[0] = 0.0
    k = int(np.argmax(Sk))
    return {"k_peak": k, "S_peak": float(Sk[k])}


def small_f64(torch, sclbm):
    """The plain FP64 case: 64x64 periodic, caption couplings, A = rho0 = 0.7,
    tau = 1, seed 1, 1000 steps (its parity with the oracle is a test)."""
    sim = sclbm.Simulation(64, 64, storage="f64", tiling="auto", **WORKLOAD)
    sim.init_random(1)
    m0 = sim.diagnostics()["mass"]
    steps = 1000
    ms, _ = timed(torch, lambda: sim.step(steps))
    d = sim.diagnostics()
    step_s = ms * 1e-3 / steps
    out = {"workload": "64x64 periodic FP64, caption couplings, A=rho0=0.7, tau=1, seed 1",
           "steps": steps, "us_per_step": round(step_s * 1e6, 3),
           "mlups": round(64 * 64 / step_s / 1e6, 1),
           "mass_drift": [float(abs(d["mass"][s] / m0[s] - 1.0)) for s in (0, 1)],
           "tiling": list(sim.get_tiling())}
    sim.close()
    log(f"small f64: {out}")
    return out


def rho0_sweep(a, torch, sclbm, head):
    out = []
    for rho0 in (0.60, 0.70, 0.75):
        row = {"rho0": rho0}
        for storage in ("f32", "f64"):
            if storage == a.storage and rho0 == a.rho0 and head is not None:
                sim, ms, d = head
            else:
                sim, ms, _, d = run_gpu(a.nx, storage, a.steps, a.warmup, rho0, 1000, torch,
                                        sclbm)
            row[storage] = {
                "mlups": round(a.nx * a.nx * a.steps / (ms * 1e-3) / 1e6, 1),
                "mass_drift": [float(abs(d["mass"][s] / d["mass0"][s] - 1.0)) for s in (0, 1)],
                "nonfinite_sites": int(d["bad_sites"]),
                **structure_peak(torch, sim)}
            if sim is not (head[0] if head else None):
                sim.close()
        out.append(row)
        log(f"sweep rho0={rho0}: {row}")
    return {"steps": a.warmup + a.steps, "reference": "FP64 GPU path (matches the oracle to 1e-10 "
            "at 1000 steps; trajectories decorrelate later, so peaks are compared)",
            "runs": out}


def sheared_cell(a, torch, sclbm):
    """1024x1024 two-species cell between a resting bottom wall and a top wall
    moving at U, random start: mean shear stress on the moving wall over the
    last 10% of the steps, and the apparent viscosity of the final state and
    of the row profiles averaged over 10 samples of those steps.  FP64 from
    several seeds gives the run-to-run spread of these observables; FP32 and
    FP16 deviation storage (stochastic rounding, and round-to-nearest for
    comparison) from seed 1 are read against FP64 seed 1 and that spread.
    Also the plain fluid (G = 0) started from rest, against Stokes' first
    problem, in every storage."""
    from paper_0807_4471_amd.observables import (apparent_viscosity, mean_wall_stress,
                                                 shear_observables, shear_profiles)
    import numpy as np
    n, steps = 1024, a.shear_steps
    last = max(1, steps // 10)
    nsamp = 10

    def one(storage, seed, U, nx=n, ny=n, kw=None, rho=None):
        sim = sclbm.Simulation(nx, ny, storage=storage, boundary="walls", wall_u=(0.0, U),
                               rho_ref=(0.7, 0.7), tiling="auto", **(kw or WORKLOAD))
        if rho is None:
            sim.init_random(seed)
        else:
            sim.init_fields(rho)
        ms, _ = timed(torch, lambda: sim.step(steps - last))
        sim.reset_wall_accum()
        # the last steps in nsamp pieces, the row profiles read after each:
        # their average gives a time-averaged apparent viscosity beside the
        # final snapshot's
        prof = []
        for k in range(nsamp):
            sim.step(last // nsamp + (1 if k < last % nsamp else 0))
            if rho is None:
                prof.append(shear_profiles(sim))
        obs = shear_observables(sim) if rho is None else \
            {"wall_stress": mean_wall_stress(sim.diagnostics(), nx)}
        if rho is None:
            ux = np.mean([p[0] for p in prof], axis=0)
            sxy = np.mean([p[1] for p in prof], axis=0)
            obs["eta_app_avg"] = apparent_viscosity(ux, sxy, float(np.mean([p[2] for p in prof])))[0]
        obs["mlups"] = round(nx * ny * (steps - last) / (ms * 1e-3) / 1e6, 1)
        sim.close()
        return obs

    runs = []
    for U in (0.01, 0.05, 0.1):
        row = {"U": U}
        ens = [one("f64", seed, U) for seed in range(1, a.shear_seeds + 1)]
        row["f64"] = ens[0]
        st = np.array([o["wall_stress"] for o in ens])
        et = np.array([o["eta_app"] for o in ens])
        ea = np.array([o["eta_app_avg"] for o in ens])
        row["f64_seed_spread"] = {
            "seeds": len(ens), "wall_stress": [float(v) for v in st],
            "wall_stress_mean": float(st.mean()), "wall_stress_sd": float(st.std(ddof=1)),
            "wall_stress_rel_sd": float(st.std(ddof=1) / abs(st.mean())),
            "eta_app_mean": float(et.mean()), "eta_app_sd": float(et.std(ddof=1)),
            "eta_app_avg_mean": float(ea.mean()), "eta_app_avg_sd": float(ea.std(ddof=1))}
        for storage in ("f32", "f16sr", "f16dev"):
            obs = one(storage, 1, U)
            for k, sd in (("wall_stress", row["f64_seed_spread"]["wall_stress_sd"]),
                          ("eta_app", row["f64_seed_spread"]["eta_app_sd"]),
                          ("eta_app_avg", row["f64_seed_spread"]["eta_app_avg_sd"])):
                d = abs(obs[k] - row["f64"][k])
                obs[k + "_rel_err"] = d / abs(row["f64"][k])
                obs[k + "_within_seed_spread"] = bool(d <= sd)
            row[storage] = obs
        runs.append(row)
        log(f"shear U={U}: {row}")
    # plain fluid started from rest: Stokes' first problem (64 columns stand
    # for the x-uniform flow), stress over the same last steps
    U, nx = 0.1, 64
    t = np.arange(steps - last, steps) + 0.5
    nu = (1.0 - 0.5) / 3.0
    stokes = 1.4 * U * math.sqrt(nu / math.pi) * float(np.mean(1.0 / np.sqrt(t)))
    g0 = dict(Ga=(0.0, 0.0), Gr=(0.0, 0.0), Gx=0.0, rho0=0.7)
    plain = {"workload": f"G = 0, {nx}x{n} channel at rest, top wall at U = {U}, {steps} steps",
             "stokes_wall_stress": stokes}
    for storage in ("f64", "f32", "f16sr", "f16dev"):
        o = one(storage, 0, U, nx=nx, kw=g0, rho=np.full((2, n, nx), 0.7))
        plain[storage] = {"wall_stress": o["wall_stress"],
                          "rel_err_vs_stokes": abs(o["wall_stress"] / stokes - 1.0)}
    log(f"shear, plain fluid: {plain}")
    torch.cuda.empty_cache()
    return {"workload": f"{n}x{n} sheared cell, top wall at U, caption couplings, rho0=0.70, "
                        f"5% random start, {steps} steps; stress over the last {last}",
            "reference": "FP64 GPU path (matches the oracle to <= 1e-9 in both observables on "
                         "128x64 x 2000 steps); the FP64 seeds give the run-to-run spread of the "
                         "observables, against which the FP32/FP16 differences from FP64 seed 1 "
                         "are read.  f16sr: FP16 deviations rounded stochastically (the FP16 "
                         "storage of this workload); f16dev: rounded to nearest, which is biased "
                         "in steady wall-driven flow (see plain_fluid)",
            "runs": runs, "plain_fluid": plain}


def rheology(a, torch, sclbm):
    """The shear-flow experiment of the paper's rheology part: 128x128
    periodic, Kolmogorov body force rho_s F0 sin(2 pi y / 128) with
    F0 = nu0 k^2 U0, U0 = 0.1 (a plain fluid would reach R = 1), Psi
    amplitude sqrt(rho0) as in the paper, random start; the response
    R(t) = u_bar / U0 and the interface indicator I_AB(t) from the fused FP64
    diagnostics (FP32 storage unless --rheology-storage says otherwise).
    Both coupling sets the paper prints are run: the one listed with the
    rheology experiment (G^r_A = 11.80, G^a_B = -11.70) and the Fig. 2
    caption set (G^r_A = 11.70, G^a_B = -11.80), each with the Shan-Chen
    velocity shift and with Guo forcing."""
    import math
    n, U0, rho0 = 128, 0.1, 0.7
    nu0 = (1.0 - 0.5) / 3.0
    F0 = nu0 * (2 * math.pi / n) ** 2 * U0
    text = dict(Ga=(-12.55, -11.70), Gr=(11.80, 10.95))
    caption = dict(Ga=(-12.55, -11.80), Gr=(11.70, 10.95))
    sets = {"rheology_text": (text, "shift"), "fig2_caption": (caption, "shift"),
            "rheology_text_guo": (text, "guo"), "fig2_caption_guo": (caption, "guo")}
    out = {"workload": f"{n}x{n} Kolmogorov flow, U0={U0}, F0={F0:.3e}, G_AB=0.58, "
                       "Psi amplitude sqrt(rho0), rho0=0.7, tau=1, 5% random start, "
                       f"{a.rheology_storage} storage, fused diagnostics every 1000 steps",
           "runs": {}}
    for name, (cp, forcing) in sets.items():
        sim = sclbm.Simulation(n, n, storage=a.rheology_storage, diag_every=1000,
                               tiling="auto", Gx=0.58, rho0=rho0, psi_amp=math.sqrt(rho0),
                               body_F0=F0, forcing=forcing, **cp)
        sim.init_random(1)
        chunk = max(1000, a.rheology_steps // 20)
        samples, t_ms, steps = [], 0.0, 0
        while steps < a.rheology_steps:
            k = min(chunk, a.rheology_steps - steps)
            ms, _ = timed(torch, lambda: sim.step(k))
            t_ms += ms
            steps += k
            sim.step(1)               # its first launch reduces the state at t = steps
            d = sim.fused_diagnostics()
            samples.append({"t": int(d["step"]), "R": round(d["u_bar"] / U0, 5),
                            "I_AB": round(d["i_ab"], 2), "bad_sites": int(d["bad_sites"])})
        sim.close()
        rs = [x["R"] for x in samples]
        out["runs"][name] = {"couplings": cp, "forcing": forcing, "steps": steps,
                             "mlups": round(n * n * steps / (t_ms * 1e-3) / 1e6, 1),
                             "R_min": min(rs), "R_final": rs[-1], "samples": samples}
        log(f"rheology {name}: R_min {min(rs)}, R_final {rs[-1]}")
    return out


def ageing(a, torch, sclbm):
    """The ageing experiment (Eq. (CORRE)): an ensemble of 128x128 lattices
    under the Kolmogorov force (U0 = 0.02, and 0.03 for one waiting time),
    couplings and Psi amplitude of the rheology experiment, seeds 1..M,
    advanced together as one batch; the overlap
    C(t_w, tau) = sum_k sum_r phi_k(t_w) phi_k(t_w + tau) / sum_k sum_r phi_k(t_w)^2
    of phi = rho_A - rho_B, from FP64 sums taken by the library's order-
    parameter pass against the snapshots phi_k(t_w)."""
    import math
    n, rho0 = 128, 0.7
    nu0 = (1.0 - 0.5) / 3.0
    taus = [0, 1000, 3000, 10000, 30000, 100000, 200000, 300000]
    out = {"workload": f"ensemble of {a.ageing_members} x {n}x{n} Kolmogorov flows, "
                       "couplings of the rheology experiment, Psi amplitude sqrt(rho0), "
                       "rho0=0.7, tau=1, 5% random starts (seeds 1..M), FP32, one batch",
           "runs": []}
    for U0, tws in ((0.02, [50000, 200000, 300000]), (0.03, [300000])):
        F0 = nu0 * (2 * math.pi / n) ** 2 * U0
        kw = dict(Ga=(-12.55, -11.70), Gr=(11.80, 10.95), Gx=0.58, rho0=rho0,
                  psi_amp=math.sqrt(rho0), body_F0=F0)
        sims = [sclbm.Simulation(n, n, storage="f32", **kw).init_random(1 + k)
                for k in range(a.ageing_members)]
        b = sclbm.Batch(sims, "auto")
        events = sorted(set(tws) | {tw + tau for tw in tws for tau in taus})
        snaps, den, C = {}, {}, {tw: {} for tw in tws}
        t, ms_total = 0, 0.0
        for T in events:
            if T > t:
                ms, _ = timed(torch, lambda: b.step(T - t))
                ms_total += ms
                t = T
            if T in tws:
                snaps[T] = [torch.empty((n, n), dtype=torch.float64, device=sims[0].buf.device)
                            for _ in sims]
                den[T] = sum(s.order_parameter(phi_out=p)[1] for s, p in zip(sims, snaps[T]))
            for tw in snaps:
                if T - tw in taus:
                    num = sum(s.order_parameter(phi_ref=p)[0] for s, p in zip(sims, snaps[tw]))
                    C[tw][T - tw] = round(num / den[tw], 6)
        b.close()
        bad = sum(1 for s in sims if s.diagnostics()["bad_sites"] > 0)
        for s in sims:
            s.close()
        run = {"U0": U0, "steps": t, "members_with_bad_sites": bad,
               "batched_mlups": round(len(sims) * n * n * t / (ms_total * 1e-3) / 1e6, 1),
               "C": {str(tw): {str(k): v for k, v in sorted(C[tw].items())} for tw in tws}}
        out["runs"].append(run)
        log(f"ageing U0={U0}: {run}")
    torch.cuda.empty_cache()
    return out


def laplace_sweep(a, torch, sclbm):
    """Nominal surface tension against rho0 (the Laplace test behind Fig. 2,
    left): static droplets of A in B on 64x64 periodic lattices, radii
    8..20, rho0 from 0.55 to 0.80, both Psi amplitudes (rho0 and
    sqrt(rho0)), caption couplings, FP64, all droplets advanced together as
    one batch; sigma and the intercept from dP = sigma / R + c0, with dP
    from the bulk pressure of the relaxed density fields."""
    import math
    from paper_0807_4471_amd import inputs
    from paper_0807_4471_amd.observables import droplet_jump, laplace_fit
    L, radii = 64, (8.0, 11.0, 14.0, 17.0, 20.0)
    rho0s = (0.55, 0.60, 0.65, 0.70, 0.72, 0.75, 0.80)
    cases, sims = [], []
    for amp_name in ("rho0", "sqrt_rho0"):
        for r0 in rho0s:
            amp = r0 if amp_name == "rho0" else math.sqrt(r0)
            params = dict(Ga=(-12.55, -11.80), Gr=(11.70, 10.95), Gx=0.58, rho0=r0, psi_amp=amp)
            for R in radii:
                sims.append(sclbm.Simulation(L, L, storage="f64", forcing=a.laplace_forcing,
                                             **params).init_fields(
                    inputs.droplet_densities(L, L, R, 1.5, 0.06)))
                cases.append((amp_name, r0, R, params))
    b = sclbm.Batch(sims, "auto")
    ms, _ = timed(torch, lambda: b.step(a.laplace_steps))
    b.close()
    pts = {}
    for (amp_name, r0, R, params), sim in zip(cases, sims):
        m = sim.moments()
        pts.setdefault((amp_name, r0), []).append(droplet_jump(m["rhoA"], m["rhoB"], params))
        sim.close()
    out = {"workload": f"{len(sims)} static droplets on {L}x{L} (radii {radii}), caption "
                       f"couplings, FP64, {a.laplace_forcing} forcing, {a.laplace_steps} "
                       "steps in one batch",
           "batched_mlups": round(len(sims) * L * L * a.laplace_steps / (ms * 1e-3) / 1e6, 1),
           "sigma": {}}
    def num(v, k):
        return round(v, k) if math.isfinite(v) else None

    for (amp_name, r0), p in pts.items():
        sigma, c0, r2 = laplace_fit([x[0] for x in p], [x[1] for x in p])
        good = [x for x in p if math.isfinite(x[1])]
        # a sigma is quoted only where the droplets reached a Laplace state
        # (dP linear in 1/R); otherwise the fit is reported without it
        law = math.isfinite(r2) and r2 >= 0.99
        out["sigma"].setdefault(amp_name, {})[str(r0)] = {
            "sigma": num(sigma, 5) if law else None, "c0": num(c0, 6) if law else None,
            "r2": num(r2, 5), "laplace_state": bool(law), "droplets_kept": len(good),
            "dP_max": num(max((x[1] for x in good), default=float("nan")), 6)}
    out["interface_stability"] = interface_stability(torch, sclbm)
    log(f"laplace: {out['sigma']}")
    log(f"interface stability: {out['interface_stability']}")
    return out


def interface_stability(torch, sclbm):
    """Sign of the surface tension from a flat interface: a slab of A in B
    with a varicose ripple (128x128, 20k steps, FP32, all in one batch) for
    both Psi amplitudes over rho0.  sigma > 0 relaxes it to two flat
    interfaces (2 crossings of phi = 0 per column along y, none along x);
    sigma < 0 breaks it into a growing micro-structure."""
    import math
    from paper_0807_4471_amd import inputs
    from paper_0807_4471_amd.observables import interface_crossings
    L, steps = 128, 20000
    rho = inputs.ripple_slab_densities(L, L, 1.2, 0.2)
    cases = [(amp, r0) for amp in ("rho0", "sqrt_rho0")
             for r0 in (0.50, 0.55, 0.60, 0.65, 0.70, 0.72, 0.75, 0.80)]
    sims = [sclbm.Simulation(L, L, storage="f32", Ga=(-12.55, -11.80), Gr=(11.70, 10.95),
                             Gx=0.58, rho0=r0, psi_amp=r0 if amp == "rho0" else math.sqrt(r0))
            .init_fields(rho) for amp, r0 in cases]
    b = sclbm.Batch(sims, "auto")
    b.step(steps)
    b.close()
    out = {"workload": f"rippled slab {L}x{L}, caption couplings, FP32, {steps} steps"}
    for (amp, r0), s in zip(cases, sims):
        m = s.moments()
        cy, cx = interface_crossings(m["rhoA"], m["rhoB"])
        out.setdefault(amp, {})[str(r0)] = {
            "crossings_y": cy, "crossings_x": cx, "flat": bool((cy, cx) == (2 * L, 0)),
            "bad_sites": s.diagnostics()["bad_sites"]}
        s.close()
    torch.cuda.empty_cache()
    return out


def run_batch(a, torch, sclbm):
    from paper_0807_4471_amd.inputs import batch_mix
    mix = batch_mix()
    sites = sum(m["nx"] * m["ny"] for m in mix)

    def make(tiling=None, subset=None):
        sims = []
        for i, m in enumerate(mix):
            if subset is not None and i not in subset:
                continue
            kw = dict(WORKLOAD, rho0=m["rho0"], Gx=m["Gx"], tau=m["tau"])
            s = sclbm.Simulation(m["nx"], m["ny"], storage="f32", tiling=tiling, **kw)
            s.init_random(m["seed"])
            sims.append(s)
        return sims

    sims = make()
    b = sclbm.Batch(sims, "auto")
    info = b.info()
    ms_b, _ = timed(torch, lambda: b.step(a.batch_steps))
    b.status()
    # the same instances, continued for the same number of steps in one
    # persistent cooperative launch (its own best tuned policy), or again
    # step-wise (untimed) when that mode is left out, so that they end where
    # the instances run one at a time below end
    info_p, ms_p = None, None
    if "persistent" not in a.batch_modes.split(","):
        b.step(a.batch_steps)
        b.status()
    b.close()
    if "persistent" in a.batch_modes.split(","):
        from paper_0807_4471_amd import autotune
        tl_p, _ = autotune.batch_plan(sims, mode="persistent")
        bp = sclbm.Batch(sims, tl_p, mode="persistent")
        info_p = bp.info()
        ms_p, _ = timed(torch, lambda: bp.step(a.batch_steps))
        bp.status()
        bp.close()
    seq = make(tiling="auto")
    ms_s, _ = timed(torch, lambda: [s.step(a.batch_steps) for s in seq])
    ms_s2, _ = timed(torch, lambda: [s.step(a.batch_steps) for s in seq])
    same = all(torch.equal(x.buf[:x.nbytes], y.buf[:y.nbytes]) for x, y in zip(sims, seq))
    # instances whose densities left the physical range (non-positive sites;
    # the method under these readings with tau_s < 1, recorded by the oracle
    # for the 128^2 members): reported apart, and the healthy ones timed again
    # as a batch of their own
    bad_sites = [s.diagnostics()["bad_sites"] for s in sims]
    diverged = [i for i, b in enumerate(bad_sites) if b > 0]
    healthy = [i for i, b in enumerate(bad_sites) if b == 0]
    for s in sims + seq:
        s.close()
    del sims, seq
    torch.cuda.empty_cache()
    hs = make(subset=healthy)
    bh = sclbm.Batch(hs, "auto")
    ms_h, _ = timed(torch, lambda: bh.step(a.batch_steps))
    bh.status()
    bh.close()
    h_sites = sum(mix[i]["nx"] * mix[i]["ny"] for i in healthy)
    for s in hs:
        s.close()
    del hs
    torch.cuda.empty_cache()
    lups = sites * a.batch_steps
    out = {"workload": "64 uneven FP32 instances (128^2..512^2, rho0~U(0.6,0.8), "
                       "G^X~U(0.5,0.65), tau_s~U(0.8,1.2)) advanced together, tuned "
                       "batch policy; each instance also run alone for comparison",
           "instances": len(mix), "sites": sites, "steps": a.batch_steps,
           "batched_mlups": round(lups / (ms_b * 1e-3) / 1e6, 1),
           "persistent_launch_mlups": round(lups / (ms_p * 1e-3) / 1e6, 1) if ms_p else None,
           "sequential_mlups": round(2 * lups / ((ms_s + ms_s2) * 1e-3) / 1e6, 1),
           "speedup": round((ms_s + ms_s2) / 2 / ms_b, 3),
           "bitwise_equal_to_sequential": bool(same),
           "instances_with_bad_sites": len(diverged),
           "diverged": {"instances": diverged, "bad_sites": [bad_sites[i] for i in diverged],
                        "share_of_sites": round(1.0 - h_sites / sites, 4),
                        "note": "densities left the physical range (non-positive sites, "
                                "guarded and counted by the kernels); every such instance "
                                "has a tau_s < 1 (velocity-shift coupling)"},
           "healthy": {"instances": len(healthy), "sites": h_sites,
                       "batched_mlups": round(h_sites * a.batch_steps / (ms_h * 1e-3) / 1e6, 1)},
           "plan": info, "persistent_plan": info_p}
    # rooflines of the batch kernels: every site of every instance reads and
    # writes its 18 populations once per step; the counter traffic was taken
    # on the step-wise kernel over this mix
    out["roofline"] = roofline(sites, "f32", ms_b / a.batch_steps, ny=1)
    if info.get("mode") == "stepwise":
        with_traffic(out["roofline"], traffic_for("batch_f32_64"))
    if ms_p:
        out["persistent_roofline"] = roofline(sites, "f32", ms_p / a.batch_steps, ny=1)
    return out


def run_serving(a, torch, sclbm, rate_lups):
    from paper_0807_4471_amd import serving
    if a.serve_capacity_glups:
        rate_lups = a.serve_capacity_glups * 1e9
    side, steps = (64, 1024), (1000, 100000)
    e_sites = (side[1] ** 2 - side[0] ** 2) / (2.0 * math.log(side[1] / side[0]))
    e_steps = (steps[1] - steps[0]) / math.log(steps[1] / steps[0])
    rate = a.serve_load * rate_lups / (e_sites * e_steps)
    trace = serving.make_trace(a.serve_requests, rate=rate, seed=4242, side=side, steps=steps)
    legs = set(a.serve_legs.split(","))

    def progress(name):
        state = {"done": 0, "last": time.perf_counter()}

        def on_event(kind, rid, t):
            if kind != "finish":
                return
            state["done"] += 1
            now = time.perf_counter()
            if now - state["last"] > 30 or state["done"] == len(trace):
                state["last"] = now
                log(f"  {name}: {state['done']}/{len(trace)} finished at t={t:.1f} s")
        return on_event

    out = {"workload": f"{a.serve_requests} Poisson requests at {rate:.3f}/s "
                       f"(load {a.serve_load} of {rate_lups / 1e9:.1f} GLUPS), sizes 64^2..1024^2 "
                       "and steps 1e3..1e5 log-uniform, f32 or f16sr, half sheared walls",
           "arrival_rate_per_s": round(rate, 4)}
    if "step" in legs:
        out["batched"] = serving.summarize_public(
            serving.Server(keep_moments=False).run(trace, on_event=progress("step-fair")))
        log(f"serving (batched, step-fair slices): {out['batched']}")
    if "work" in legs:
        out["batched_work_fair"] = serving.summarize_public(
            serving.Server(keep_moments=False, slicing="work").run(
                trace, on_event=progress("work-fair")))
        log(f"serving (batched, work-fair slices): {out['batched_work_fair']}")
    if "seq" in legs:
        out["sequential_f64"] = serving.summarize_public(
            serving.serve_sequential_f64(trace, on_event=progress("sequential FP64")))
        log(f"serving (sequential FP64): {out['sequential_f64']}")
    return out


def cpu_threads() -> int:
    """Host threads this process may use: its CPU affinity, capped by
    OMP_NUM_THREADS when that is set (the share of a shared host)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    env = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, min(n, int(env))) if env.isdigit() and int(env) > 0 else max(1, n)


def cpu_baseline(rho0, scale: float = 1.0):
    """The FP64 oracle on the host (the same seeded 5% random start, caption
    couplings) at 64^2, 512^2 and 1024^2, single-threaded and on all the
    process's cores (OpenMP over rows; the arithmetic is the same).  Step
    counts are bounded so the whole sample is ~25 s of host time; `value` is
    the all-core rate on the headline's 512^2 lattice."""
    import numpy as np
    import oracle
    from paper_0807_4471_amd import inputs
    oracle.build(force=False)
    nthr = cpu_threads()
    runs = []
    for nx, s1, sn in ((64, 1000, 1000), (512, 150, 600), (1024, 40, 200)):
        p = oracle.Params(nx=nx, ny=nx, **dict(WORKLOAD, rho0=rho0))
        for threads, steps in ((1, s1), (nthr, sn)):
            steps = max(1, int(steps * scale))
            used = oracle.set_threads(threads)
            f = oracle.init(p, inputs.random_densities(nx, nx, 1))
            t0 = time.perf_counter()
            oracle.run(p, f, steps)
            dt = time.perf_counter() - t0
            assert np.isfinite(f).all()
            runs.append({"nx": nx, "threads": used, "steps": steps, "seconds": round(dt, 3),
                         "mlups": round(nx * nx * steps / dt / 1e6, 4)})
    oracle.set_threads(0)
    head = [r for r in runs if r["nx"] == 512][-1]
    return {"value": head["mlups"], "unit": "MLUPS", "cores": head["threads"], "kind": "oracle",
            "sample": f"FP64 oracle, {head['nx']}x{head['nx']} periodic, same couplings and "
                      f"seeded init, {head['steps']} steps on {head['threads']} threads "
                      f"({head['seconds']} s); also 1 thread and 64^2, 1024^2 in runs "
                      f"(host: {host_cpu()})",
            "runs": runs}


def host_cpu() -> str:
    """Model name of the host CPU, with the number of cores the OS shows."""
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}, {os.cpu_count()} logical cores visible"


def calibrate_copy(torch):
    n = 1 << 30
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": 5}))


def main():
    global DEVICE_WARMUP_MS
    a = parse()
    DEVICE_WARMUP_MS = a.device_warmup_ms
    if a.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {a.gpus} is not supported "
              "(the lattice would shard into y-slabs with halo exchange; not built).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(3)
    if a.calibrate_copy:
        calibrate_copy(torch)
        return
    from paper_0807_4471_amd import sclbm
    nx, storage = a.nx, a.storage
    sim, ms_total, wall, d = run_gpu(nx, storage, a.steps, a.warmup, a.rho0, 1000, torch, sclbm,
                                     forcing=a.forcing)
    ms_step = ms_total / a.steps
    mlups = nx * nx / (ms_step * 1e-3) / 1e6
    roof = roofline(nx, storage, ms_step)
    with_traffic(roof, traffic_for(f"{storage}_{nx}" + ("_guo" if a.forcing == "guo" else "")))
    # ping-pong footprint (2 copies x 18 populations) vs the 256 MiB Infinity Cache
    roof["cache_resident"] = BYTES_PER_LUP[storage] * nx * nx < 256 * 2 ** 20
    if roof["cache_resident"]:
        roof["note"] = ("the ping-pong state fits the 256 MB Infinity Cache, so this fraction "
                        "is against the HBM peak but not bound by HBM; the HBM-roofline claims "
                        "are the DRAM-resident lattices of dram_resident")
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "f16dev": "f32 (f16 storage)",
                  "f16sr": "f32 (f16 storage)"}[storage],
        "data": "synthetic",
        "config": {"workload": f"micro-emulsion {nx}x{nx} periodic two-species D2Q9 "
                               f"Shan-Chen, {storage} populations, rho0={a.rho0}, "
                               "A=rho0, caption couplings, tau=1, 5% random init"
                               + (", Guo forcing" if a.forcing == "guo" else ""),
                   "nx": nx, "ny": nx, "storage": storage, "diag_every": 1000,
                   "forcing": a.forcing,
                   "tiling": list(sim.get_tiling())},
        "roofline": roof,
        "mass_drift": [float(abs(d["mass"][s] / d["mass0"][s] - 1.0)) for s in (0, 1)],
        "wall_s": round(wall, 3),
        "device_warmup": {"ms": a.device_warmup_ms,
                          "what": "after the warmup steps, the step kernel runs on a scratch "
                                  "lattice of the same shape for this long before the timed "
                                  "region; the timed lattice gets exactly `warmup` steps"},
    }
    log(f"headline: {out['value']} MLUPS, {roof['kernel_us']} us/step, frac {roof['frac']}")
    if not a.no_sweep:
        out["rho0_sweep"] = rho0_sweep(a, torch, sclbm, (sim, ms_total, d))
    # run-to-run spread: five more timed regions of 20k steps on the same
    # lattice (after the sweep has read its state)
    if a.repeats > 0:
        reps = sorted(timed(torch, lambda: sim.step(20000))[0] / 20000 for _ in range(a.repeats))
        out["repeats"] = {"runs": a.repeats, "steps_each": 20000,
                          "median_us_per_step": round(reps[len(reps) // 2] * 1e3, 3),
                          "min_us_per_step": round(reps[0] * 1e3, 3),
                          "max_us_per_step": round(reps[-1] * 1e3, 3)}
        log(f"headline repeats: {out['repeats']}")
    sim.close()
    del sim
    torch.cuda.empty_cache()
    if not a.no_guo:
        other = "guo" if a.forcing == "shift" else "shift"
        k = max(1000, a.steps // 5)
        s2, mt, _, d2 = run_gpu(nx, storage, k, a.warmup, a.rho0, 1000, torch, sclbm,
                                forcing=other)
        r = roofline(nx, storage, mt / k)
        out["forcing_variant"] = {
            "forcing": other, "steps": k, "mlups": round(nx * nx / (mt / k * 1e-3) / 1e6, 1),
            "ms_per_step": round(mt / k, 6), "frac": r["frac"],
            "mass_drift": [float(abs(d2["mass"][q] / d2["mass0"][q] - 1.0)) for q in (0, 1)]}
        log(f"forcing variant: {out['forcing_variant']}")
        s2.close()
        del s2
        torch.cuda.empty_cache()
    if not a.no_small:
        out["small_f64"] = small_f64(torch, sclbm)
    if not a.no_dram:
        side = []
        for st_, n_, m_ in (("f32", 4096, 4096), ("f16dev", 4096, 4096), ("f16sr", 4096, 4096),
                            ("f64", 2048, 2048), ("f32", 8192, 1024), ("f16dev", 8192, 1024)):
            s2, mt, _, _ = run_gpu(n_, st_, 200, 20, a.rho0, 0, torch, sclbm, ny=m_)
            r = roofline(n_, st_, mt / 200, ny=m_)
            with_traffic(r, traffic_for(f"{st_}_{n_}" if n_ == m_ else f"{st_}_{n_}x{m_}"))
            what = "(DRAM-resident)" if n_ == m_ else \
                "(one GPU's slab of a lattice split by rows, DRAM-resident)"
            side.append({"workload": f"{n_}x{m_} {st_} {what}",
                         "mlups": round(n_ * m_ / (mt / 200 * 1e-3) / 1e6, 1), "roofline": r,
                         "tiling": list(s2.get_tiling())})
            log(f"dram: {side[-1]}")
            s2.close()
            del s2
            torch.cuda.empty_cache()
        out["dram_resident"] = side
    if not a.no_shear:
        out["sheared_cell"] = sheared_cell(a, torch, sclbm)
    if not a.no_rheology:
        out["rheology"] = rheology(a, torch, sclbm)
    if not a.no_ageing:
        out["ageing"] = ageing(a, torch, sclbm)
    if not a.no_laplace:
        out["laplace"] = laplace_sweep(a, torch, sclbm)
    rate_lups = 2.0e10
    if not a.no_batch:
        out["batch"] = run_batch(a, torch, sclbm)
        rate_lups = out["batch"]["batched_mlups"] * 1e6
    if not a.no_serve:
        out["serving"] = run_serving(a, torch, sclbm, rate_lups)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a.rho0, a.cpu_scale)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
