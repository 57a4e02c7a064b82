"""The allocation-free batch entry point (sclbm_batch_step_static, the
batch tables in the library's static device array) against the existing
batch path (sclbm_batch_plan + sclbm_batch_step, STEPWISE, tables in a
caller workspace): bitwise equal results on two calls in a row, the second
with a smaller batch, so the second call runs on what the first left in the
array."""
import numpy as np
import pytest

from helpers import WORKLOAD, banner

pytestmark = pytest.mark.gpu

FIRST = [  # nx, ny, boundary, extra, tiling, steps
    (200, 200, "periodic", {}, (50, 4, 4, 1), 23),
    (130, 50, "walls", dict(wall_u=(0.0, 0.05)), (130, 16, 4, 0), 17),
    (300, 37, "periodic", dict(tau=(0.9, 1.1)), (252, 8, 4, 0, 1), 30),
    (57, 200, "walls", dict(wall_u=(-0.02, 0.03)), (57, 4, 4, 1), 11),
    (96, 96, "periodic", dict(forcing="guo"), (48, 4, 4, 1), 0),
]
SECOND = [
    (40, 30, "periodic", {}, (40, 4, 4, 1), 9),
    (64, 20, "walls", dict(wall_u=(0.0, 0.1)), (64, 5, 4, 0), 14),
]


def _sims(storage, cases, seed0):
    from paper_0807_4471_amd import sclbm
    out = []
    for k, (nx, ny, bnd, extra, _, _) in enumerate(cases):
        s = sclbm.Simulation(nx, ny, storage=storage, boundary=bnd, **{**WORKLOAD, **extra})
        s.init_random(seed0 + k)
        out.append(s)
    return out


@pytest.mark.parametrize("storage", ["f32", "f16sr", "f64"])
def test_static_batch_equals_workspace_batch(storage):
    from paper_0807_4471_amd import sclbm
    for call, cases in enumerate((FIRST, SECOND)):
        banner(f"{storage} static-scratch batch, call {call + 1} ({len(cases)} instances)")
        seed0 = 500 + 10 * call
        a = _sims(storage, cases, seed0)
        b = _sims(storage, cases, seed0)
        tilings = [c[4] for c in cases]
        steps = [c[5] for c in cases]
        sclbm.batch_step_static(a, tilings, steps)
        ref = sclbm.Batch(b, tilings, mode="stepwise")
        ref.step(steps)
        ref.close()
        for k, (x, y) in enumerate(zip(a, b)):
            assert x.t == y.t == steps[k]
            mx, my = x.moments(), y.moments()
            for key in ("rhoA", "rhoB", "ux", "uy"):
                assert np.array_equal(mx[key], my[key]), (call, k, key)
            if cases[k][2] == "walls":
                assert np.array_equal(x.diagnostics()["wall_mom"], y.diagnostics()["wall_mom"])
        for s in a + b:
            s.close()
