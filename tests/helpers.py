"""Shared helpers for the GPU tests: run the same seeded input through the
HIP library (via its C ABI binding) and through the CPU oracle."""
from __future__ import annotations

import numpy as np

import oracle
from paper_0807_4471_amd import inputs

WORKLOAD = dict(Ga=(-12.55, -11.80), Gr=(11.70, 10.95), Gx=0.58, rho0=0.70)
_ORACLE_KEYS = ("tau", "Ga", "Gr", "Gx", "rho0", "psi_amp", "wall_u", "body_F0", "forcing")


def banner(msg: str):
    print(f"[case] {msg}", flush=True)


def gpu_run(nx, ny, steps, rho=None, ux=None, uy=None, seed=1, tiling=None, **kw):
    """Returns (Simulation, moments dict) after `steps` steps.  tiling: None
    (library default), "auto" (the tuned table, as the benchmark runs) or a
    tuple."""
    from paper_0807_4471_amd import sclbm
    sim = sclbm.Simulation(nx, ny, tiling="auto" if tiling == "auto" else None, **kw)
    if tiling is not None and tiling != "auto":
        sim.set_tiling(*tiling)
    if rho is None:
        rho = inputs.random_densities(nx, ny, seed)
    sim.init_fields(rho, ux, uy)
    sim.step(steps)
    return sim, sim.moments()


def oracle_run(nx, ny, steps, rho=None, ux=None, uy=None, seed=1, boundary="periodic", **kw):
    """Returns (params, f, (rho, ux, uy)) of the FP64 oracle."""
    okw = {k: v for k, v in kw.items() if k in _ORACLE_KEYS}
    p = oracle.Params(nx=nx, ny=ny, walls=(boundary == "walls"), **okw)
    if rho is None:
        rho = inputs.random_densities(nx, ny, seed)
    f = oracle.init(p, rho, ux, uy)
    oracle.run(p, f, steps)
    return p, f, oracle.moments(p, f)


def max_err(m: dict, ref) -> dict:
    r, ux, uy = ref
    return {
        "rho": max(np.abs(m["rhoA"] - r[0]).max(), np.abs(m["rhoB"] - r[1]).max()),
        "u": max(np.abs(m["ux"] - ux).max(), np.abs(m["uy"] - uy).max()),
    }


def structure_factor(phi: np.ndarray):
    """Radially averaged S(k) of phi - <phi> on integer |k| shells; returns
    (k_shell, S) with S normalised by the number of sites."""
    ny, nx = phi.shape
    F = np.fft.fft2(phi - phi.mean())
    S = (np.abs(F) ** 2) / (nx * ny)
    ky = np.fft.fftfreq(ny) * ny
    kx = np.fft.fftfreq(nx) * nx
    K = np.sqrt(ky[:, None] ** 2 + kx[None, :] ** 2)
    shell = np.rint(K).astype(int)
    nsh = shell.max() + 1
    tot = np.bincount(shell.ravel(), S.ravel(), nsh)
    cnt = np.bincount(shell.ravel(), None, nsh)
    ks = np.arange(nsh)
    ok = cnt > 0
    return ks[ok][1:], (tot[ok] / cnt[ok])[1:]


def window_half_width(steps: int) -> int:
    """Half-width of a periodic window whose centre evolves exactly as on the
    full lattice for `steps` steps and whose velocity read-out is exact: one
    step reaches 1 site (streaming) + 2 sites (the 25-point Psi stencil),
    the read-out adds the force stencil (2), plus one site of margin."""
    return 3 * steps + 2 + 1


def oracle_window_moments(nx, ny, seed, sites, steps, mean=(0.7, 0.7), amp=0.05, **kw):
    """Oracle (rho_A, rho_B, u_x, u_y) at `sites` [(y, x), ...] of the periodic
    nx x ny lattice initialised by inputs.random_densities(nx, ny, seed),
    after `steps` steps, each from a periodic window around the site."""
    okw = {k: v for k, v in kw.items() if k in _ORACLE_KEYS}
    h = window_half_width(steps)
    w = 2 * h + 1
    p = oracle.Params(nx=w, ny=w, **okw)
    out = []
    for (y, x) in sites:
        ys = np.arange(y - h, y + h + 1) % ny
        xs = np.arange(x - h, x + h + 1) % nx
        rho = inputs.random_densities_window(nx, ny, seed, ys, xs, mean, amp)
        f = oracle.init(p, rho)
        oracle.run(p, f, steps)
        r, ux, uy = oracle.moments(p, f)
        out.append((r[0][h, h], r[1][h, h], ux[h, h], uy[h, h]))
    return np.array(out)


def oracle_column_moments(nx, ny, seed, columns, steps, boundary="walls", mean=(0.7, 0.7),
                          amp=0.05, **kw):
    """Oracle (rho_A, rho_B, u_x, u_y) of whole columns x in `columns` of the
    nx x ny lattice (walls or periodic in y) started from
    inputs.random_densities(nx, ny, seed), after `steps` steps, each from a
    full-height window periodic in x around the column (exact for the
    centre column by the same reach argument as the square windows).
    Returns an array [len(columns), 4, ny]."""
    okw = {k: v for k, v in kw.items() if k in _ORACLE_KEYS}
    h = window_half_width(steps)
    w = 2 * h + 1
    p = oracle.Params(nx=w, ny=ny, walls=(boundary == "walls"), **okw)
    out = []
    for x in columns:
        xs = np.arange(x - h, x + h + 1) % nx
        rho = inputs.random_densities_window(nx, ny, seed, np.arange(ny), xs, mean, amp)
        f = oracle.init(p, rho)
        oracle.run(p, f, steps)
        r, ux, uy = oracle.moments(p, f)
        out.append(np.stack([r[0][:, h], r[1][:, h], ux[:, h], uy[:, h]]))
    return np.array(out)


# One-step rounding bounds of the stored densities (max |drho| after one
# step against the FP64 oracle), derived from the storage arithmetic: a
# density is a sum of 9 stored populations, FP32 rounds values <= 0.5 to
# <= 2^-25 each (9 * 2^-25 ~ 3e-7, plus the FP32 collision of the same
# order); binary16 deviations |h| <= ~0.03 have ulp 2^-16, so <= 9 * 2^-17 ~
# 7e-5 per step.  Rounded up to 1e-6 and 1.5e-4.  FP64: the same sum in
# binary64 (9 * 2^-54 ~ 5e-16) plus a few hundred operations of the step,
# each rounded to 2^-53 relative on values of order one, taken in a
# different order (and with fused multiply-adds) on the GPU: 1e-14.
ONE_STEP = {"f64": 1e-14, "f32": 1e-6, "f16dev": 1.5e-4, "f16sr": 1.5e-4}


def oracle_amplification(nx, ny, steps, seed=1, rho=None, boundary="periodic", eps=1e-9,
                         with_moments=False, **kw):
    """Envelope A(m), m = 0..steps, of the growth of a small density
    perturbation over m steps of this case, measured on the oracle: the
    initial densities are perturbed by at most eps (a seeded +-pattern), both
    runs advance step by step, and A(m) is the largest ratio max|drho(k)| /
    max|drho(0)| for k <= m (so it is non-decreasing, and >= 1).  With
    with_moments, also returns the unperturbed run's final moments (those of
    oracle_run on the same case)."""
    okw = {k: v for k, v in kw.items() if k in _ORACLE_KEYS}
    p = oracle.Params(nx=nx, ny=ny, walls=(boundary == "walls"), **okw)
    if rho is None:
        rho = inputs.random_densities(nx, ny, seed)
    pert = eps * inputs.uniform_pm1(seed + 7919, np.arange(2 * nx * ny)).reshape(2, ny, nx)
    f0 = oracle.init(p, rho)
    f1 = oracle.init(p, rho + pert)
    d0 = np.abs(oracle.moments(p, f1)[0] - oracle.moments(p, f0)[0]).max()
    amp = np.ones(steps + 1)
    d = d0
    for m in range(1, steps + 1):
        oracle.run(p, f0, 1)
        oracle.run(p, f1, 1)
        d = np.abs(oracle.moments(p, f1)[0] - oracle.moments(p, f0)[0]).max()
        amp[m] = max(amp[m - 1], d / d0)
    # the envelope is a linear-response bound: valid only while the grown
    # perturbation is still small against the fields themselves
    if d > 1e-3:
        raise ValueError(f"perturbation grew to {d:.3g}: nonlinear, no rounding bound from it")
    if with_moments:
        return amp, oracle.moments(p, f0)
    return amp


def accumulated_bound(storage, amp, steps):
    """Bound on max |drho| after `steps` steps in reduced-precision storage:
    the stored initial state and every step each add at most
    ONE_STEP[storage], and an error made k steps before the end grows at
    most by the envelope A(k) (oracle_amplification), so the sum is
    ONE_STEP * sum_{k <= steps} A(k).  A factor 2 covers rounding of
    populations that leaves the density unchanged (momentum, stress) and may
    grow differently from a density perturbation."""
    return 2.0 * ONE_STEP[storage] * float(np.sum(amp[:steps + 1]))
