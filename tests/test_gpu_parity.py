"""FP64 parity of the HIP path (through the C ABI) against the CPU oracle.

Bar: the workload's 64x64 FP64 case must match to <= 1e-10 max-abs density
after 1000 steps.  Shorter runs are held to 1e-12 (FP64 rounding of a few
hundred operations per value, amplified at most ~1e3x by the demixing
transient; measured ~1e-15 per step).  Sizes span several strips and
chunks with ragged tails, odd shapes, lattices narrower than one strip and
shorter than the stencil.
"""
import numpy as np
import pytest

from helpers import (WORKLOAD, accumulated_bound, banner, gpu_run, max_err, oracle_amplification,
                     oracle_run)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nx,ny,steps", [
    (1, 1, 3), (2, 3, 5), (5, 5, 10), (8, 8, 20), (9, 7, 20), (13, 21, 25),
    (64, 1, 10), (1, 40, 10), (70, 37, 30), (125, 19, 15), (300, 45, 8),
])
def test_small_and_ragged_f64(nx, ny, steps):
    banner(f"f64 periodic {nx}x{ny} steps={steps}")
    _, m = gpu_run(nx, ny, steps, storage="f64", **WORKLOAD)
    _, _, ref = oracle_run(nx, ny, steps, **WORKLOAD)
    e = max_err(m, ref)
    assert e["rho"] <= 1e-12 and e["u"] <= 1e-12, e


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_workload_64_f64_1000_steps(seed):
    """64x64, FP64, tau = 1, A = rho0 = 0.7, the caption couplings, 1000 steps."""
    banner(f"f64 64x64 1000 steps seed={seed}")
    _, m = gpu_run(64, 64, 1000, seed=seed, storage="f64", **WORKLOAD)
    _, _, ref = oracle_run(64, 64, 1000, seed=seed, **WORKLOAD)
    e = max_err(m, ref)
    assert e["rho"] <= 1e-10, e
    assert ref[0].shape == (2, 64, 64)


@pytest.mark.parametrize("variant", ["sqrt_amp", "text_couplings", "unequal_tau", "gx_only"])
def test_parameter_variants_f64(variant):
    kw = dict(WORKLOAD)
    if variant == "sqrt_amp":
        kw["psi_amp"] = 0.7 ** 0.5
    elif variant == "text_couplings":
        kw.update(Ga=(-12.55, -11.70), Gr=(11.80, 10.95))
    elif variant == "unequal_tau":
        kw["tau"] = (0.8, 1.25)
    else:
        kw.update(Ga=(0.0, 0.0), Gr=(0.0, 0.0), Gx=1.2)
    banner(f"f64 variant {variant}")
    _, m = gpu_run(48, 40, 60, storage="f64", **kw)
    _, _, ref = oracle_run(48, 40, 60, **kw)
    e = max_err(m, ref)
    assert e["rho"] <= 1e-12 and e["u"] <= 1e-12, e


@pytest.mark.parametrize("nx,ny,uw", [(40, 24, (0.0, 0.05)), (67, 9, (-0.03, 0.1)),
                                      (5, 2, (0.02, 0.0)), (130, 50, (0.0, 0.1))])
def test_walls_f64(nx, ny, uw):
    banner(f"f64 walls {nx}x{ny} wall_u={uw}")
    sim, m = gpu_run(nx, ny, 120, storage="f64", boundary="walls", wall_u=uw, **WORKLOAD)
    p, f, ref = oracle_run(nx, ny, 120, boundary="walls", wall_u=uw, **WORKLOAD)
    e = max_err(m, ref)
    assert e["rho"] <= 1e-11 and e["u"] <= 1e-12, e


def test_wall_momentum_f64():
    import oracle
    from paper_0807_4471_amd import inputs, sclbm
    nx, ny, uw = 36, 20, (0.0, 0.08)
    banner("f64 wall momentum exchange")
    rho = inputs.random_densities(nx, ny, 4)
    sim = sclbm.Simulation(nx, ny, storage="f64", boundary="walls", wall_u=uw, **WORKLOAD)
    sim.init_fields(rho)
    sim.step(50)
    sim.reset_wall_accum()
    sim.step(30)
    d = sim.diagnostics()
    p = oracle.Params(nx=nx, ny=ny, walls=True, wall_u=uw, **WORKLOAD)
    f = oracle.init(p, rho)
    oracle.run(p, f, 50)
    wm = np.zeros((2, 2))
    oracle.run(p, f, 30, wm)
    assert d["wall_steps"] == 30
    np.testing.assert_allclose(d["wall_mom"], wm, rtol=1e-9, atol=1e-12)


def test_body_force_f64():
    kw = dict(WORKLOAD, body_F0=2e-4)
    banner("f64 Kolmogorov body force")
    _, m = gpu_run(32, 48, 80, storage="f64", **kw)
    _, _, ref = oracle_run(32, 48, 80, **kw)
    e = max_err(m, ref)
    assert e["rho"] <= 1e-12 and e["u"] <= 1e-12, e


def test_moments_and_stress_f64():
    import oracle
    banner("f64 moments + sigma_xy + totals")
    sim, m = gpu_run(50, 30, 40, storage="f64", tau=(0.9, 1.1), **WORKLOAD)
    p, f, ref = oracle_run(50, 30, 40, tau=(0.9, 1.1), **WORKLOAD)
    ux_row, sxy_row = oracle.row_profiles(p, f)
    np.testing.assert_allclose(m["sxy"].mean(axis=1), sxy_row, rtol=0, atol=1e-13)
    np.testing.assert_allclose(m["ux"].mean(axis=1), ux_row, rtol=0, atol=1e-13)
    d = sim.diagnostics()
    tot = oracle.totals(p, f)
    np.testing.assert_allclose(d["mass"], tot["mass"], rtol=1e-13)
    np.testing.assert_allclose(d["mom"], tot["mom"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(d["sxy"], tot["sxy"], rtol=0, atol=1e-11)
    assert d["bad_sites"] == tot["bad"] == 0
    assert d["step"] == 40


def test_fused_diagnostics_f64():
    from paper_0807_4471_amd import inputs, sclbm
    import oracle
    banner("f64 fused diagnostics every 7 steps")
    rho = inputs.random_densities(33, 29, 6)
    sim = sclbm.Simulation(33, 29, storage="f64", diag_every=7, **WORKLOAD)
    sim.init_fields(rho)
    sim.step(23)
    d = sim.fused_diagnostics()
    assert d["step"] == 21
    p = oracle.Params(nx=33, ny=29, **WORKLOAD)
    f = oracle.init(p, rho)
    oracle.run(p, f, 21)
    tot = oracle.totals(p, f)
    np.testing.assert_allclose(d["mass"], tot["mass"], rtol=1e-13)
    np.testing.assert_allclose(d["mom"], tot["mom"], rtol=0, atol=1e-12)


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 2e-5), ("f16dev", 2e-3)])
@pytest.mark.parametrize("boundary", ["periodic", "walls"])
def test_shear_flow_observables(storage, tol, boundary):
    """u_bar (Kolmogorov-mode projection of the physical velocity) and I_AB,
    on-demand and fused, against the oracle: a demixing mixture driven by
    the Kolmogorov force (and, with walls, sheared), tilings of both kinds."""
    from paper_0807_4471_amd import inputs, sclbm
    import oracle
    banner(f"{storage} {boundary} u_bar and I_AB")
    nx, ny, steps = 70, 48, 60
    kw = dict(WORKLOAD, body_F0=2e-5)
    if boundary == "walls":
        kw["wall_u"] = (0.0, 0.04)
    rho = inputs.random_densities(nx, ny, 9)
    p = oracle.Params(nx=nx, ny=ny, walls=boundary == "walls",
                      **{k: v for k, v in kw.items() if k in ("Ga", "Gr", "Gx", "rho0",
                                                               "body_F0", "wall_u")})
    f = oracle.init(p, rho)
    oracle.run(p, f, steps)
    ref = oracle.shear_flow(p, f)
    assert abs(ref["u_bar"]) > 1e-6 and abs(ref["i_ab"]) > 1e-6
    for tl in [(60, 4, 4, 1), (70, 16, 2, 0)]:
        sim = sclbm.Simulation(nx, ny, storage=storage, boundary=boundary, diag_every=steps,
                               **kw)
        sim.set_tiling(*tl)
        sim.init_fields(rho)
        sim.step(steps)
        on_demand = sim.diagnostics()             # state at t = steps
        sim.step(1)                               # its first kernel reduces t = steps
        fused = sim.fused_diagnostics()
        assert fused["step"] == on_demand["step"] == steps
        for name, d in (("on-demand", on_demand), ("fused", fused)):
            for k in ("u_bar", "i_ab"):
                err = abs(d[k] - ref[k]) / abs(ref[k])
                print(f"  {tl} {name} {k}: {d[k]:.12e} vs {ref[k]:.12e} (rel {err:.1e})",
                      flush=True)
        for name, d in (("on-demand", on_demand), ("fused", fused)):
            for k in ("u_bar", "i_ab"):
                assert abs(d[k] - ref[k]) <= tol * abs(ref[k]), (tl, name, k, d[k], ref[k])
        sim.close()


def test_init_random_matches_input_generator():
    """The device SplitMix64 init equals the host generator bit for bit."""
    from paper_0807_4471_amd import inputs, sclbm
    banner("init_random vs inputs.random_densities")
    nx, ny = 77, 45
    a = sclbm.Simulation(nx, ny, storage="f64").init_random(12345, mean=(0.7, 0.65), amp=0.05)
    b = sclbm.Simulation(nx, ny, storage="f64")
    b.init_fields(inputs.random_densities(nx, ny, 12345, mean=(0.7, 0.65), amp=0.05))
    ma, mb = a.moments(), b.moments()
    for k in ("rhoA", "rhoB", "ux", "uy"):
        assert np.array_equal(ma[k], mb[k]), k
    r = inputs.random_densities(nx, ny, 12345, mean=(0.7, 0.65), amp=0.05)
    assert np.abs(ma["rhoA"] - r[0]).max() < 1e-15
    a.step(5)
    b.step(5)
    assert np.array_equal(a.moments()["rhoA"], b.moments()["rhoA"])


def test_init_with_velocity_f64():
    rng = np.random.default_rng(3)
    nx, ny = 31, 26
    ux = 0.03 * rng.standard_normal((ny, nx))
    uy = 0.03 * rng.standard_normal((ny, nx))
    banner("f64 init with velocity field")
    _, m = gpu_run(nx, ny, 15, ux=ux, uy=uy, storage="f64", **WORKLOAD)
    _, _, ref = oracle_run(nx, ny, 15, ux=ux, uy=uy, **WORKLOAD)
    e = max_err(m, ref)
    assert e["rho"] <= 1e-12 and e["u"] <= 1e-12, e


@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev", "f16sr"])
@pytest.mark.parametrize("ny", [2, 3, 4, 5, 9])
@pytest.mark.parametrize("tiling", [None, (7, 4, 4, 1), (7, 8, 8, 1), (7, 4, 1, 0)])
def test_walls_short_lattices_all_tilings(storage, ny, tiling):
    """Walls on lattices no taller than a stacked tile: every staged row must
    fold into the lattice (regression: rows beyond one mirror image)."""
    nx = 7
    kw = dict(WORKLOAD, boundary="walls", wall_u=(0.01, 0.04))
    banner(f"{storage} walls {nx}x{ny} tiling={tiling}")
    _, m = gpu_run(nx, ny, 12, storage=storage, tiling=tiling, **kw)
    _, _, ref = oracle_run(nx, ny, 12, **kw)
    e = max_err(m, ref)
    if storage == "f64":
        tol = 1e-12
    else:   # one-step bound summed over the steps, amplified as the oracle measures
        tol = accumulated_bound(storage, oracle_amplification(nx, ny, 12, **kw), 12)
    assert e["rho"] <= tol, (e, tol)


@pytest.mark.parametrize("case", ["workload", "unequal_tau", "body_force", "walls"])
def test_guo_forcing_f64(case):
    """Guo forcing (barycentric velocity with half the force, source term
    (1 - 1/(2 tau)) w_i [3 (c_i - u).F + 9 (c_i.u)(c_i.F)]) against the oracle."""
    kw = dict(WORKLOAD, forcing="guo")
    nx, ny, steps, bound = 48, 40, 60, "periodic"
    if case == "unequal_tau":
        kw["tau"] = (0.8, 1.25)
    elif case == "body_force":
        kw["body_F0"] = 2e-4
    elif case == "walls":
        bound, kw["wall_u"] = "walls", (0.0, 0.06)
    banner(f"f64 guo {case}")
    _, m = gpu_run(nx, ny, steps, storage="f64", boundary=bound, **kw)
    _, _, ref = oracle_run(nx, ny, steps, boundary=bound, **kw)
    e = max_err(m, ref)
    print(f"  guo {case}: {e}", flush=True)
    assert e["rho"] <= 1e-12 and e["u"] <= 1e-12, e
    # the two couplings differ on this workload (the test would pass vacuously
    # if the flag were ignored)
    _, _, shift = oracle_run(nx, ny, steps, boundary=bound,
                             **{k: v for k, v in kw.items() if k != "forcing"})
    assert max_err(m, shift)["rho"] > 1e-6


def test_guo_forcing_workload_1000_steps_f64():
    banner("f64 guo 64x64 1000 steps")
    _, m = gpu_run(64, 64, 1000, storage="f64", forcing="guo", **WORKLOAD)
    _, _, ref = oracle_run(64, 64, 1000, forcing="guo", **WORKLOAD)
    e = max_err(m, ref)
    print(f"  guo 1000 steps: {e}", flush=True)
    assert e["rho"] <= 1e-10, e


@pytest.mark.parametrize("storage,tol", [("f32", 1e-6), ("f16dev", 1.5e-4), ("f16sr", 1.5e-4)])
@pytest.mark.parametrize("tiling", [None, (60, 4, 4, 1), (70, 16, 2, 0)])
def test_guo_forcing_reduced_precision_one_step(storage, tol, tiling):
    """One step in reduced-precision storage, both kernel families: the same
    one-step bounds as the shift coupling."""
    banner(f"{storage} guo one step tiling={tiling}")
    _, m = gpu_run(130, 70, 1, storage=storage, tiling=tiling, forcing="guo", **WORKLOAD)
    _, _, ref = oracle_run(130, 70, 1, forcing="guo", **WORKLOAD)
    e = max_err(m, ref)
    print(f"  guo one step {storage}: {e}", flush=True)
    assert e["rho"] <= tol, e


def test_guo_forcing_batch_matches_single():
    """A batch of Guo and shift instances steps each like its single run."""
    from paper_0807_4471_amd import inputs, sclbm
    banner("f32 guo + shift batch")
    shapes = [(64, 48, "guo"), (100, 30, "shift"), (33, 65, "guo")]
    singles, members = [], []
    for i, (nx, ny, fc) in enumerate(shapes):
        rho = inputs.random_densities(nx, ny, 20 + i)
        for lst in (singles, members):
            s = sclbm.Simulation(nx, ny, storage="f32", forcing=fc, **WORKLOAD)
            s.init_fields(rho)
            lst.append(s)
    for s in singles:
        s.step(25)
    b = sclbm.Batch(members)
    b.step(25)
    for s, t in zip(singles, members):
        a, c = s.moments(), t.moments()
        for k in ("rhoA", "rhoB", "ux", "uy"):
            assert np.array_equal(a[k], c[k]), k
    b.close()
