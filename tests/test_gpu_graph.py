"""Steps captured in a HIP graph: `sclbm_step` only enqueues kernel launches,
so a caller may capture an even number of steps and replay them.  Each
replay, with eager library and torch work and synchronisations between the
replays, must leave exactly the state that the same number of eager steps
leaves (FP64 and FP32: bitwise; periodic and walls, with fused
diagnostics), and the eager result is pinned to the FP64 oracle."""
import numpy as np
import pytest

from helpers import WORKLOAD, accumulated_bound, banner, max_err, oracle_amplification, oracle_run
from paper_0807_4471_amd import inputs

pytestmark = pytest.mark.gpu

K = 4          # steps per captured graph (even: the ping-pong copy comes back)
REPLAYS = 3


@pytest.mark.parametrize("storage,boundary", [("f64", "periodic"), ("f32", "periodic"),
                                              ("f32", "walls")])
def test_graph_replays_equal_eager_steps(storage, boundary):
    import torch
    from paper_0807_4471_amd import sclbm
    banner(f"graph capture of {K} steps, {REPLAYS} replays, {storage} {boundary}")
    nx, ny, warm = 96, 72, 10
    kw = dict(WORKLOAD, storage=storage, boundary=boundary, diag_every=2)
    if boundary == "walls":
        kw["wall_u"] = (0.0, 0.05)
    rho = inputs.random_densities(nx, ny, 5)

    ref = sclbm.Simulation(nx, ny, **kw)
    ref.init_fields(rho)
    ref.step(warm)
    got = sclbm.Simulation(nx, ny, **kw)
    got.init_fields(rho)
    got.step(warm)

    side = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            got.step(K)          # recorded, not run
    torch.cuda.synchronize()
    scratch = torch.zeros(1 << 16, device="cuda")
    for r in range(REPLAYS):
        g.replay()
        # eager work of the program between replays
        scratch.add_(1.0)
        torch.cuda.synchronize()
        ref.step(K)
        a, b = ref.moments(), got.moments()
        for k in ("rhoA", "rhoB", "ux", "uy"):
            assert np.array_equal(a[k], b[k]), (r, k)
    assert float(scratch[0]) == REPLAYS

    # the eager path itself against the oracle after the same number of steps
    total = warm + K * REPLAYS
    okw = dict(WORKLOAD)
    if boundary == "walls":
        okw["wall_u"] = (0.0, 0.05)
    _, _, want = oracle_run(nx, ny, total, rho=rho, boundary=boundary, **okw)
    e = max_err(ref.moments(), want)
    if storage == "f64":
        tol = 1e-12
    else:
        amp = oracle_amplification(nx, ny, total, rho=rho, boundary=boundary, **okw)
        tol = accumulated_bound(storage, amp, total)
    print(f"  eager vs oracle after {total} steps: {e}, bound {tol:.3g}", flush=True)
    assert e["rho"] <= tol and e["u"] <= tol
    ref.close()
    got.close()
