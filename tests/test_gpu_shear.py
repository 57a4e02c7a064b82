"""Shear observables of the sheared two-species cell (moving top wall) on the
GPU, in every storage, against the FP64 oracle: mean shear stress on the
moving wall over the last steps, and the apparent viscosity from the
row-mean stress and shear-rate profiles.  The oracle side computes both from
its own wall-momentum accumulator and row profiles, with the definitions
written out here."""
import numpy as np
import pytest

import oracle
from helpers import WORKLOAD, banner
from paper_0807_4471_amd import inputs

pytestmark = pytest.mark.gpu

NX, NY, STEPS, LAST = 128, 64, 2000, 500
# Relative tolerances (stress, viscosity).  FP64 differs from the oracle by
# rounding order and exp only (measured <= 2.1e-11).  In FP32 and FP16 the
# error is rounding amplified by the demixing dynamics (a 1-ulp change of the
# initial state grows by orders of magnitude within 1000 steps), which the
# arithmetic alone does not bound: the tolerances are 3x the largest error
# measured over U in {0.01, 0.05, 0.1} (FP32 5.0e-4 / 4.5e-3, FP16
# deviations 3.2e-2 / 2.2e-2, FP16 with stochastic rounding of every
# population 5.5e-2 / -).  The latter's apparent viscosity from one final
# snapshot is dominated by its rounding noise at the lowest shear (measured
# relative error 1.1 at U = 0.01): it is reported, not asserted.
TOL = {"f64": (1e-9, 1e-9), "f32": (1.5e-3, 1.5e-2), "f16dev": (0.1, 0.07),
       "f16sr": (0.17, None)}


def oracle_observables(U, seed):
    p = oracle.Params(nx=NX, ny=NY, walls=True, wall_u=(0.0, U), **WORKLOAD)
    f = oracle.init(p, inputs.random_densities(NX, NY, seed))
    oracle.run(p, f, STEPS - LAST)
    wm = np.zeros((2, 2))
    oracle.run(p, f, LAST, wm)
    stress = -wm[1, 0] / (NX * LAST)
    ux_row, sxy_row = oracle.row_profiles(p, f)
    rho, _, _ = oracle.moments(p, f)
    g = 0.5 * (ux_row[2:] - ux_row[:-2])
    s = sxy_row[1:-1]
    m = np.abs(g) > 0.01 * np.abs(g).max()
    eta = float(np.sum(s[m] * g[m]) / np.sum(g[m] ** 2))
    return stress, eta, float(rho.sum(axis=0).mean())


def gpu_observables(U, seed, storage):
    from paper_0807_4471_amd import sclbm
    from paper_0807_4471_amd.observables import shear_observables
    sim = sclbm.Simulation(NX, NY, storage=storage, boundary="walls", wall_u=(0.0, U),
                           rho_ref=(0.7, 0.7), **WORKLOAD)
    sim.init_random(seed)
    sim.step(STEPS - LAST)
    sim.reset_wall_accum()
    sim.step(LAST)
    out = shear_observables(sim)
    sim.close()
    return out


_ref_cache = {}


@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev", "f16sr"])
@pytest.mark.parametrize("U", [0.01, 0.05, 0.1])
def test_shear_observables_against_oracle(U, storage):
    banner(f"sheared cell {NX}x{NY} U={U} {storage} {STEPS} steps")
    if U not in _ref_cache:
        _ref_cache[U] = oracle_observables(U, seed=11)
    s_ref, eta_ref, rho_mean = _ref_cache[U]
    got = gpu_observables(U, 11, storage)
    e_s = abs(got["wall_stress"] - s_ref) / abs(s_ref)
    e_eta = abs(got["eta_app"] - eta_ref) / abs(eta_ref)
    print(f"  stress {got['wall_stress']:.9e} vs {s_ref:.9e} (rel {e_s:.2e}); "
          f"eta {got['eta_app']:.9e} vs {eta_ref:.9e} (rel {e_eta:.2e})", flush=True)
    assert got["wall_steps"] == LAST and got["bad_sites"] == 0
    tol_s, tol_eta = TOL[storage]
    assert e_s <= tol_s
    if tol_eta is not None:
        assert e_eta <= tol_eta
