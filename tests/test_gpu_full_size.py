"""Parity at the workload sizes, in the launch configuration the benchmark
times (default tiling of the library / the tuned tiling)."""
import numpy as np
import pytest

from helpers import WORKLOAD, banner, gpu_run, max_err, oracle_run

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("rho0", [0.60, 0.70, 0.75])
def test_512_f32_all_sites(rho0):
    """512x512 FP32 (the micro-emulsion workload), every site after 10 steps."""
    kw = dict(WORKLOAD, rho0=rho0)
    banner(f"f32 512x512 rho0={rho0} 10 steps")
    _, m = gpu_run(512, 512, 10, storage="f32", **kw)
    _, _, ref = oracle_run(512, 512, 10, **kw)
    e = max_err(m, ref)
    print(f"  512^2 f32 error: {e}", flush=True)
    assert e["rho"] <= 10 * 1e-6, e


def test_512_f64_all_sites():
    banner("f64 512x512 20 steps")
    _, m = gpu_run(512, 512, 20, storage="f64", **WORKLOAD)
    _, _, ref = oracle_run(512, 512, 20, **WORKLOAD)
    e = max_err(m, ref)
    assert e["rho"] <= 1e-13, e


@pytest.mark.parametrize("U", [0.01, 0.1])
def test_1024_walls_f16dev(U):
    """1024x1024 sheared cell, FP16 deviation storage, 3 steps, every site."""
    kw = dict(WORKLOAD, boundary="walls", wall_u=(0.0, U))
    banner(f"f16dev 1024x1024 walls U={U} 3 steps")
    _, m = gpu_run(1024, 1024, 3, storage="f16dev", rho_ref=(0.7, 0.7), **kw)
    _, _, ref = oracle_run(1024, 1024, 3, **kw)
    e = max_err(m, ref)
    print(f"  1024^2 f16dev walls error: {e}", flush=True)
    assert e["rho"] <= 3 * 1.5e-4, e


@pytest.mark.parametrize("storage", ["f32", "f16dev"])
def test_4096_uniform_fixed_point(storage):
    """Largest bench lattice: a uniform state stays uniform (any size).  FP32
    keeps it bit for bit.  FP16 deviation storage rounds the rest population
    stochastically, so sites differ by at most a few units of the deviation's
    binary16 ulp (|h| <= 4/9 * 0.05 -> ulp 2^-16) per step."""
    from paper_0807_4471_amd import sclbm
    banner(f"{storage} 4096x4096 uniform state")
    n = 4096
    s = sclbm.Simulation(n, n, storage=storage, **WORKLOAD)
    s.init_random(1, mean=(0.7, 0.65), amp=0.0)
    s.step(3)
    m = s.moments_device()
    for k, v in (("rhoA", 0.7), ("rhoB", 0.65)):
        t = m[k]
        spread = float(t.max() - t.min())
        if storage == "f32":
            assert spread == 0.0
        else:
            assert spread <= 3 * 4 * 2.0 ** -16, spread
        assert abs(float(t.mean()) - v) < (1e-6 if storage == "f32" else 1e-4)
    if storage == "f32":
        assert float(m["ux"].abs().max()) == 0.0
    else:
        assert float(m["ux"].abs().max()) < 1e-4
