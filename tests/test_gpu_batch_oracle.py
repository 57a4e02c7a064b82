"""Batched launches against the FP64 oracle: every member of an uneven batch
(sizes, periodic and moving walls, unequal tau, Guo forcing, a body force),
in both execution modes and every storage type, element by element.

FP64 members must match the oracle to 1e-12 (the bar of the short-run FP64
parity tests).  FP32 and FP16 members must match within the accumulated
rounding bound of helpers.accumulated_bound: the storage's one-step bound
summed over the steps, each step's error amplified at most by the growth
the oracle measures for a perturbation of the same case."""
import numpy as np
import pytest

from helpers import (WORKLOAD, accumulated_bound, banner, max_err, oracle_amplification,
                     oracle_run)

pytestmark = pytest.mark.gpu

CASES = [  # nx, ny, boundary, extra parameters
    (64, 64, "periodic", {}),
    (100, 70, "periodic", dict(tau=(0.9, 1.1))),
    (192, 192, "periodic", dict(rho0=0.65, Gx=0.6)),
    (130, 50, "walls", dict(wall_u=(0.0, 0.05))),
    (300, 37, "periodic", {}),
    (57, 200, "walls", dict(wall_u=(-0.02, 0.03))),
    (80, 60, "periodic", dict(forcing="guo", tau=(0.85, 1.2))),
    (96, 48, "periodic", dict(body_F0=2e-5)),
]
STEPS = [30, 17, 30, 5, 0, 22, 25, 19]
TILINGS = [(60, 4, 4, 1), (100, 8, 4, 0, 1), (60, 4, 4, 1), (130, 16, 4, 0), (252, 8, 4, 0, 1),
           (57, 4, 4, 1), (40, 12, 4, 0), (48, 4, 4, 1)]
SEED0 = 70

_ref = {}


def _oracle(k):
    if k not in _ref:
        nx, ny, bnd, extra = CASES[k]
        kw = {**WORKLOAD, **extra}
        _, _, mom = oracle_run(nx, ny, STEPS[k], seed=SEED0 + k, boundary=bnd, **kw)
        amp = oracle_amplification(nx, ny, STEPS[k], seed=SEED0 + k, boundary=bnd, **kw)
        _ref[k] = (mom, amp)
    return _ref[k]


@pytest.mark.parametrize("mode", ["persistent", "stepwise"])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev", "f16sr"])
def test_batch_members_match_oracle(storage, mode):
    from paper_0807_4471_amd import sclbm
    banner(f"{storage} {mode} batch of {len(CASES)} vs FP64 oracle")
    sims = []
    for k, (nx, ny, bnd, extra) in enumerate(CASES):
        s = sclbm.Simulation(nx, ny, storage=storage, boundary=bnd, **{**WORKLOAD, **extra})
        s.init_random(SEED0 + k)
        sims.append(s)
    b = sclbm.Batch(sims, TILINGS, mode=mode)
    b.step(STEPS)
    b.status()
    for k, s in enumerate(sims):
        mom, amp = _oracle(k)
        e = max_err(s.moments(), mom)
        tol = 1e-12 if storage == "f64" else accumulated_bound(storage, amp, STEPS[k])
        print(f"  member {k} {CASES[k][:3]} steps={STEPS[k]}: err {e}, bound {tol:.3g}",
              flush=True)
        assert s.t == STEPS[k]
        assert e["rho"] <= tol and e["u"] <= tol, (k, e, tol)
    b.close()
