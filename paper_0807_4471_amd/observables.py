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


def shear_observables(sim) -> dict:
    """Wall stress and apparent viscosity of a walls Simulation (syncs)."""
    d = sim.diagnostics()
    m = sim.moments()
    ux_row = m["ux"].mean(axis=1)
    sxy_row = m["sxy"].mean(axis=1)
    rho_mean = float((m["rhoA"] + m["rhoB"]).mean())
    eta, nu = apparent_viscosity(ux_row, sxy_row, rho_mean)
    return {"wall_stress": mean_wall_stress(d, sim.nx), "eta_app": eta, "nu_app": nu,
            "wall_steps": int(d["wall_steps"]), "bad_sites": int(d["bad_sites"])}
