"""Batched launches (one persistent launch per call, or one ordinary launch
per step): uneven instances advanced together must give bit-for-bit the
results of stepping each alone (same per-site arithmetic, same rounding
keys), for every storage type, boundary, tiling and mode."""
import numpy as np
import pytest

from helpers import WORKLOAD, banner

pytestmark = pytest.mark.gpu

CASES = [  # nx, ny, boundary, extra
    (64, 64, "periodic", {}),
    (100, 70, "periodic", dict(tau=(0.9, 1.1))),
    (192, 192, "periodic", dict(rho0=0.65, Gx=0.6)),
    (130, 50, "walls", dict(wall_u=(0.0, 0.05))),
    (300, 37, "periodic", {}),
    (57, 200, "walls", dict(wall_u=(-0.02, 0.03))),
]


def _make(storage, nx, ny, boundary, extra, seed):
    from paper_0807_4471_amd import sclbm
    kw = dict(WORKLOAD)
    kw.update(extra)
    s = sclbm.Simulation(nx, ny, storage=storage, boundary=boundary, **kw)
    s.init_random(seed)
    return s


@pytest.mark.parametrize("mode", ["persistent", "stepwise"])
@pytest.mark.parametrize("storage", ["f32", "f16dev", "f16sr", "f64"])
def test_batch_equals_alone_bitwise(storage, mode):
    from paper_0807_4471_amd import sclbm
    banner(f"{storage} {mode} batch of {len(CASES)} vs alone")
    steps = [30, 17, 30, 5, 0, 22]
    tilings = [(60, 4, 4, 1), (100, 8, 4, 0, 1), (60, 4, 4, 1), (130, 16, 4, 0), (252, 8, 4, 0, 1),
               (57, 4, 4, 1)]
    batch_sims = [_make(storage, *c, seed=10 + k) for k, c in enumerate(CASES)]
    b = sclbm.Batch(batch_sims, tilings, mode=mode)
    b.step(steps)
    b.status()
    for k, c in enumerate(CASES):
        alone = _make(storage, *c, seed=10 + k)
        alone.step(steps[k])
        ma, mb = alone.moments(), batch_sims[k].moments()
        assert batch_sims[k].t == steps[k]
        for key in ("rhoA", "rhoB", "ux", "uy"):
            assert np.array_equal(ma[key], mb[key]), (k, key)


@pytest.mark.parametrize("mode", ["persistent", "stepwise"])
def test_batch_repeated_launches_and_default_tilings(mode):
    from paper_0807_4471_amd import sclbm
    banner(f"f32 {mode} batch: three launches, default tilings")
    sims = [_make("f32", *c, seed=40 + k) for k, c in enumerate(CASES)]
    b = sclbm.Batch(sims, mode=mode)
    for st in ([7, 3, 0, 7, 1, 2], [8, 8, 8, 8, 8, 8], [1, 0, 2, 0, 3, 0]):
        b.step(st)
    b.status()
    tot = [16, 11, 10, 15, 12, 10]
    for k, c in enumerate(CASES):
        alone = _make("f32", *c, seed=40 + k)
        alone.step(tot[k])
        assert sims[k].t == tot[k]
        assert np.array_equal(alone.moments()["rhoA"], sims[k].moments()["rhoA"]), k


def test_batch_wall_momentum_matches_alone():
    from paper_0807_4471_amd import sclbm
    banner("f64 batch wall momentum")
    c = (80, 40, "walls", dict(wall_u=(0.0, 0.08)))
    a = _make("f64", *c, seed=3)
    b_sim = _make("f64", *c, seed=3)
    other = _make("f64", 96, 96, "periodic", {}, seed=4)
    a.step(25)
    sclbm.Batch([b_sim, other], mode="stepwise").step([25, 40])
    da, db = a.diagnostics(), b_sim.diagnostics()
    assert np.array_equal(da["wall_mom"], db["wall_mom"])
    assert da["wall_steps"] == db["wall_steps"] == 25


def test_batch_rejects_bad_plans():
    from paper_0807_4471_amd import sclbm
    banner("batch validation")
    a = _make("f32", 64, 64, "periodic", {}, 1)
    f = _make("f64", 64, 64, "periodic", {}, 1)
    with pytest.raises(sclbm.SclbmError):
        sclbm.Batch([a, f])                       # mixed storage
    with pytest.raises(sclbm.SclbmError):
        sclbm.Batch([a], [(60, 8, 2, 0)])          # waves != 4
    with pytest.raises(sclbm.SclbmError):
        sclbm.Batch([a], [(61, 4, 4, 1)])          # stacked tile too wide


def test_barrier_time_out_is_reported_and_recoverable():
    """Force the persistent mode's grid-barrier time-out from the host (a
    limit of one sleep, while the uneven instances make workgroups wait
    microseconds): every workgroup still leaves the kernel, the batch
    reports EDEVICE, and with the default limit restored the next launch
    gives the results of running alone."""
    from paper_0807_4471_amd import sclbm
    banner("persistent batch: forced barrier time-out, then recovery")
    cases = CASES + [(768, 768, "periodic", {})]   # many more tiles than workgroups
    sims = [_make("f32", *c, seed=60 + k) for k, c in enumerate(cases)]
    b = sclbm.Batch(sims, mode="persistent")
    info = b.info()
    assert info["tiles"] > 2 * info["grid"], info
    b.set_barrier_limit(1)
    b.step([20] * len(sims))
    with pytest.raises(sclbm.SclbmError) as ei:
        b.status()
    assert ei.value.status == sclbm.EDEVICE
    b.set_barrier_limit(0)
    for k, s in enumerate(sims):
        s.init_random(60 + k)
    b.step([9] * len(sims))
    b.status()
    for k, c in enumerate(cases):
        alone = _make("f32", *c, seed=60 + k)
        alone.step(9)
        assert np.array_equal(alone.moments()["rhoA"], sims[k].moments()["rhoA"]), k
    b.close()
