"""Shear observables of the sheared two-species cell, from the FP64 read-outs
of the step kernels (wall momentum exchange, moments).

* Mean shear stress on the moving (top) wall: the x-momentum the fluid gives
  the wall, per wall node and per step, accumulated in FP64 by the kernels
  since the last `reset_wall_accum`.  A wall that drags the fluid forward
  receives negative x-momentum, so the stress the fluid exerts on the wall
  is minus this exchange; the function returns that stress.
* Apparent viscosity: the least-squares ratio of the row-mean shear stress
  sigma_xy to the local shear rate d<u_x>/dy (central differences of the
  row-mean velocity), over interior rows whose shear rate exceeds 1% of the
  largest; eta is the dynamic value, nu = eta / <rho>.
"""
from __future__ import annotations

import numpy as np


def mean_wall_stress(diag: dict, nx: int, wall: int = 1) -> float:
    """-(x-momentum exchanged with `wall`) / (nx * steps accumulated)."""
    steps = int(diag["wall_steps"])
    if steps <= 0:
        raise ValueError("no wall exchange accumulated")
    return -float(diag["wall_mom"][wall][0]) / (nx * steps)


def apparent_viscosity(ux_row: np.ndarray, sxy_row: np.ndarray, rho_mean: float):
    """(eta, nu) from row means of u_x and sigma_xy (length ny)."""
    ux_row = np.asarray(ux_row, dtype=np.float64)
    sxy_row = np.asarray(sxy_row, dtype=np.float64)
    g = 0.5 * (ux_row[2:] - ux_row[:-2])
    s = sxy_row[1:-1]
    m = np.abs(g) > 0.01 * np.abs(g).max()
    eta = float(np.sum(s[m] * g[m]) / np.sum(g[m] * g[m]))
    return eta, eta / float(rho_mean)


def shear_profiles(sim):
    """(row means of u_x, row means of sigma_xy, mean total density) of a
    walls Simulation's current state (syncs)."""
    m = sim.moments()
    return (m["ux"].mean(axis=1), m["sxy"].mean(axis=1),
            float((m["rhoA"] + m["rhoB"]).mean()))


def shear_observables(sim) -> dict:
    """Wall stress and apparent viscosity of a walls Simulation (syncs)."""
    d = sim.diagnostics()
    ux_row, sxy_row, rho_mean = shear_profiles(sim)
    eta, nu = apparent_viscosity(ux_row, sxy_row, rho_mean)
    return {"wall_stress": mean_wall_stress(d, sim.nx), "eta_app": eta, "nu_app": nu,
            "wall_steps": int(d["wall_steps"]), "bad_sites": int(d["bad_sites"])}


# ---------------------------------------------------------------- Laplace law

CS2 = 1.0 / 3.0


def bulk_pressure(rhoA, rhoB, Ga, Gr, Gx, rho0, psi_amp):
    """Bulk pressure of the two-species model at each site,
        P = c_s^2 (rho_A + rho_B) + (c_s^2 / 2) sum_s G_s1 Psi_s^2
            + c_s^2 (G_AB / rho0) rho_A rho_B,    G_s1 = G^a_s + G^r_s,
    the local part of the non-ideal pressure tensor Eq. (PAB) with the cross
    term and c_s^2 factors of the long-wave expansion of the forces."""
    rA = np.asarray(rhoA, dtype=np.float64)
    rB = np.asarray(rhoB, dtype=np.float64)
    psiA = psi_amp * (1.0 - np.exp(-rA / rho0))
    psiB = psi_amp * (1.0 - np.exp(-rB / rho0))
    g1 = (Ga[0] + Gr[0], Ga[1] + Gr[1])
    return (CS2 * (rA + rB) + 0.5 * CS2 * (g1[0] * psiA ** 2 + g1[1] * psiB ** 2)
            + CS2 * (Gx / rho0) * rA * rB)


def droplet_jump(rhoA, rhoB, params: dict, core: int = 2, min_contrast: float = 0.1):
    """(effective radius, pressure jump) of a centred droplet of species A:
    the radius from the area of A's normalised excess density, the jump
    between the mean bulk pressure of the central (2 core)^2 sites and of a
    3x3 corner block (the far field on a periodic lattice).  (nan, nan) if
    the fields are not finite or A's inside/outside contrast fell below
    min_contrast (the droplet dissolved)."""
    rA = np.asarray(rhoA, dtype=np.float64)
    ny, nx = rA.shape
    cy, cx = ny // 2, nx // 2
    a_in = rA[cy - core:cy + core, cx - core:cx + core].mean()
    a_out = rA[:3, :3].mean()
    if not (np.isfinite(rA).all() and np.isfinite(rhoB).all()) or a_in - a_out < min_contrast:
        return float("nan"), float("nan")
    radius = float(np.sqrt(np.sum((rA - a_out) / (a_in - a_out)) / np.pi))
    P = bulk_pressure(rA, rhoB, params["Ga"], params["Gr"], params["Gx"], params["rho0"],
                      params["psi_amp"])
    return radius, float(P[cy - core:cy + core, cx - core:cx + core].mean() - P[:3, :3].mean())


def laplace_fit(radii, jumps):
    """Least-squares dP = sigma / R + c0 over the finite points: (sigma, c0,
    r2), or three nans with fewer than three points."""
    R = np.asarray(radii, dtype=np.float64)
    dP = np.asarray(jumps, dtype=np.float64)
    ok = np.isfinite(R) & np.isfinite(dP)
    R, dP = R[ok], dP[ok]
    if len(R) < 3:
        return float("nan"), float("nan"), float("nan")
    M = np.vstack([1.0 / R, np.ones_like(R)]).T
    (sigma, c0), *_ = np.linalg.lstsq(M, dP, rcond=None)
    ss = np.sum((dP - dP.mean()) ** 2)
    r2 = 1.0 - np.sum((dP - M @ [sigma, c0]) ** 2) / ss if ss > 0 else 1.0
    return float(sigma), float(c0), float(r2)


# --------------------------------------------------- sign of the surface tension

def interface_crossings(rhoA, rhoB) -> tuple:
    """(crossings along y, crossings along x) of the order parameter
    phi = rho_A - rho_B: the number of neighbouring site pairs (periodic)
    whose phi differ in sign.  A flat slab has exactly 2 per column along y
    and none along x; a positive surface tension relaxes a rippled slab to
    that state, a negative one breaks it into ever more interface."""
    s = np.sign(np.asarray(rhoA, dtype=np.float64) - np.asarray(rhoB, dtype=np.float64))
    return int((s != np.roll(s, 1, axis=0)).sum()), int((s != np.roll(s, 1, axis=1)).sum())


def ripple_amplitude(rhoA, mode: int = 1) -> float:
    """Fourier coefficient on sin(2 pi mode x / nx) of the A mass per column
    (the varicose ripple of inputs.ripple_slab_densities)."""
    rA = np.asarray(rhoA, dtype=np.float64)
    nx = rA.shape[1]
    M = rA.sum(axis=0)
    return float(np.sum(M * np.sin(2.0 * np.pi * mode * np.arange(nx) / nx)) * 2.0 / nx)
