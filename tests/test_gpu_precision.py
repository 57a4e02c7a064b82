"""Reduced-precision storage (FP32; FP16 deviations f - w_i rho_ref with FP32
arithmetic) against the FP64 oracle.

Tolerances derived from the arithmetic:
  * one step: each density is a sum of 9 stored populations; FP32 rounding of
    values <= 0.5 gives <= 9 * 2^-25 ~ 3e-7 (plus the FP32 collision, same
    order); FP16 deviations |h| <= ~0.03 at 5% noise have ulp 2^-16, so
    <= 9 * 2^-17 ~ 7e-5 per step.  Tolerances: 1e-6 and 1.5e-4.
  * a stable, slowly varying flow (G = 0 shear wave) accumulates these
    errors linearly: 200 steps -> 200 x the one-step bound on the velocity
    scale of the flow.
  * in the demixing workload the uniform mixture is linearly unstable, so
    pointwise differences grow.  The pointwise bound then sums the one-step
    bound over the steps, each amplified by the growth the oracle measures
    for a small perturbation of the same run (helpers.accumulated_bound);
    over longer runs the tests compare the statistics the workloads report:
    mass (FP64 totals), structure-factor peak position and height.
"""
import numpy as np
import pytest

from helpers import ONE_STEP, WORKLOAD, banner, gpu_run, max_err, oracle_run, structure_factor

pytestmark = pytest.mark.gpu



@pytest.mark.parametrize("storage", ["f32", "f16dev", "f16sr"])
@pytest.mark.parametrize("nx,ny", [(64, 64), (130, 70)])
def test_one_step_error(storage, nx, ny):
    banner(f"{storage} one step {nx}x{ny}")
    _, m = gpu_run(nx, ny, 1, storage=storage, **WORKLOAD)
    _, _, ref = oracle_run(nx, ny, 1, **WORKLOAD)
    e = max_err(m, ref)
    print(f"  one-step error {storage}: {e}", flush=True)
    assert e["rho"] <= ONE_STEP[storage], e


@pytest.mark.parametrize("storage", ["f32", "f16dev", "f16sr"])
def test_stable_flow_accumulates_linearly(storage):
    """G = 0 shear wave, 200 steps: velocity error stays within 200 one-step
    bounds scaled by the velocity amplitude."""
    L, U = 64, 0.01
    y = np.arange(L)
    ux = np.tile((U * np.sin(2 * np.pi * y / L))[:, None], (1, L))
    rho = np.full((2, L, L), 0.7)
    kw = dict(Ga=(0.0, 0.0), Gr=(0.0, 0.0), Gx=0.0, rho0=0.7)
    banner(f"{storage} shear wave 200 steps")
    _, m = gpu_run(L, L, 200, rho=rho, ux=ux, storage=storage, **kw)
    _, _, ref = oracle_run(L, L, 200, rho=rho, ux=ux, **kw)
    e = max_err(m, ref)
    print(f"  shear-wave error {storage}: {e}", flush=True)
    assert e["rho"] <= 200 * ONE_STEP[storage] * 0.1, e
    assert e["u"] <= 200 * ONE_STEP[storage] * 0.1, e


@pytest.mark.parametrize("storage", ["f32", "f16dev", "f16sr"])
def test_demixing_workload_pointwise(storage):
    """100 steps of the 64x64 workload, every site: within the accumulated
    rounding bound (one-step bound summed over the steps, each amplified by
    the growth the oracle measures for a perturbation of this run)."""
    from helpers import accumulated_bound, oracle_amplification
    banner(f"{storage} workload 64x64 100 steps")
    _, m = gpu_run(64, 64, 100, storage=storage, **WORKLOAD)
    amp, ref = oracle_amplification(64, 64, 100, with_moments=True, **WORKLOAD)
    tol = accumulated_bound(storage, amp, 100)
    e = max_err(m, ref)
    print(f"  workload error after 100 steps {storage}: {e}, bound {tol:.3g} "
          f"(growth {amp[-1]:.3g})", flush=True)
    assert e["rho"] <= tol and e["u"] <= tol, e


@pytest.mark.parametrize("storage", ["f32", "f16dev", "f16sr"])
def test_demixing_statistics_and_mass(storage):
    """128x128, 600 steps: mass drift (FP64 totals) and S(k) of phi = rho_A -
    rho_B against the oracle."""
    from paper_0807_4471_amd import inputs
    nx = ny = 128
    banner(f"{storage} 128x128 600 steps statistics")
    sim, m = gpu_run(nx, ny, 600, storage=storage, **WORKLOAD)
    d = sim.diagnostics()
    rho0 = inputs.random_densities(nx, ny, 1)
    m0 = rho0.sum(axis=(1, 2))
    drift = np.abs(d["mass"] - m0) / m0
    print(f"  relative mass drift {storage}: {drift}", flush=True)
    assert np.all(drift < (1e-5 if storage == "f32" else 1e-3)), drift
    _, _, ref = oracle_run(nx, ny, 600, **WORKLOAD)
    kg, Sg = structure_factor(m["rhoA"] - m["rhoB"])
    ko, So = structure_factor(ref[0][0] - ref[0][1])
    kpg, kpo = kg[np.argmax(Sg)], ko[np.argmax(So)]
    print(f"  S(k) peak: gpu k={kpg} S={Sg.max():.4g}; oracle k={kpo} S={So.max():.4g}", flush=True)
    assert abs(kpg - kpo) <= 1
    assert abs(Sg.max() / So.max() - 1.0) < 0.1
    # variance of the order parameter (demixing amplitude)
    vg = (m["rhoA"] - m["rhoB"]).var()
    vo = (ref[0][0] - ref[0][1]).var()
    assert abs(vg / vo - 1.0) < 0.02


def test_f16dev_reference_density_matters():
    """Deviation storage relative to rho_ref: with rho_ref = 0 the same run
    stores full populations in binary16 and is markedly worse."""
    banner("f16dev rho_ref 0.7 vs 0")
    _, good = gpu_run(64, 64, 1, storage="f16dev", rho_ref=(0.7, 0.7), **WORKLOAD)
    _, bad = gpu_run(64, 64, 1, storage="f16dev", rho_ref=(0.0, 0.0), **WORKLOAD)
    _, _, ref = oracle_run(64, 64, 1, **WORKLOAD)
    eg, eb = max_err(good, ref)["rho"], max_err(bad, ref)["rho"]
    print(f"  f16 one-step error with/without reference: {eg:.3g} / {eb:.3g}", flush=True)
    assert eb > 5 * eg
