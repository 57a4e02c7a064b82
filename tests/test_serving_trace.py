"""Host-side pieces of the serving loop: the seeded request trace and the
latency/throughput summary (no GPU)."""
import math

import numpy as np

from paper_0807_4471_amd import serving


def test_trace_is_seeded_and_in_range():
    a = serving.make_trace(500, rate=10.0, seed=4242)
    b = serving.make_trace(500, rate=10.0, seed=4242)
    assert [(r.arrival, r.nx, r.steps, r.storage, r.boundary, r.seed) for r in a] == \
           [(r.arrival, r.nx, r.steps, r.storage, r.boundary, r.seed) for r in b]
    assert all(64 <= r.nx <= 1024 and r.nx == r.ny for r in a)
    assert all(1000 <= r.steps <= 100000 for r in a)
    assert {r.storage for r in a} == {"f32", "f16sr"}
    assert {r.boundary for r in a} == {"periodic", "walls"}
    assert all((r.wall_u in (0.01, 0.05, 0.1)) == (r.boundary == "walls") for r in a)
    arr = np.array([r.arrival for r in a])
    assert np.all(np.diff(arr) > 0)
    # Poisson: mean gap 1/rate
    assert abs(np.diff(arr).mean() - 0.1) < 0.02
    # log-uniform sizes: median near the geometric mean of the range
    assert abs(math.log(np.median([r.nx for r in a])) - math.log(256)) < 0.25


def test_summary_percentiles():
    trace = [serving.Request(rid=i, arrival=float(i), nx=10, ny=10, steps=100) for i in range(100)]
    res = {i: serving.Result(i, float(i), float(i), float(i) + 1.0 + 0.01 * i, "ok", None, None)
           for i in range(100)}
    res[5].status = "failed"
    out = serving.summarize(trace, res, makespan=200.0, busy=50.0)
    assert out["completed"] == 100 and out["failed"] == 1
    assert abs(out["p50_latency_s"] - (1.0 + 0.01 * 49.5)) < 1e-9
    assert out["p99_latency_s"] > 1.98
    assert abs(out["aggregate_mlups"] - 100 * 100 * 100 / 200.0 / 1e6) < 1e-12


def test_request_that_can_never_fit_is_rejected_not_waited_for():
    """A request whose state exceeds the whole HBM budget is refused at
    admission (status "rejected"); the loop does not wait for room that can
    never appear.  Every request here is too large, so no device work runs."""
    trace = serving.make_trace(5, rate=1e6, seed=3, side=(64, 128), steps=(10, 20))
    out = serving.Server(hbm_budget=1024).run(trace)
    assert out["rejected"] == 5 and out["completed"] == 0 and out["failed"] == 0
    assert all(r.status == "rejected" and r.moments is None for r in out["results"].values())


def test_server_parameters_are_validated():
    import pytest
    for bad in (dict(hbm_budget=0), dict(max_slots=0), dict(chunk_ms=0.0),
                dict(slicing="fifo")):
        with pytest.raises(ValueError):
            serving.Server(**bad)
