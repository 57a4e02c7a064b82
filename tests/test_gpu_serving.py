"""Continuous-batching server: requests admitted while others run, state
kept on the device, results identical (bit for bit) to running each request
alone; admission respects the HBM budget and slot limit; a corrupted request
fails alone."""
import numpy as np
import pytest

from helpers import banner

pytestmark = pytest.mark.gpu


def _trace():
    from paper_0807_4471_amd import serving
    # a short trace: arrivals close together so requests overlap on the GPU
    return serving.make_trace(14, rate=5000.0, seed=7, side=(48, 200), steps=(200, 2000))


def _alone(req):
    from paper_0807_4471_amd import serving
    sim = serving._new_sim(req, "cuda")
    sim.step(req.steps)
    return sim.moments()


@pytest.mark.parametrize("slicing", ["work", "steps"])
def test_results_equal_running_alone(slicing):
    from paper_0807_4471_amd import serving
    banner(f"serving ({slicing} slices): mix vs alone")
    trace = _trace()
    events = []
    out = serving.Server(chunk_ms=0.5, slicing=slicing).run(
        trace, on_event=lambda k, r, t: events.append((k, r, t)))
    assert out["completed"] == len(trace) and out["failed"] == 0
    # overlap: some request was admitted before an earlier one finished
    fin = {r: t for k, r, t in events if k == "finish"}
    adm = {r: t for k, r, t in events if k == "admit"}
    assert any(adm[b] < fin[a] for a in adm for b in adm if a != b and adm[a] < adm[b])
    for req in trace:
        got = out["results"][req.rid].moments
        ref = _alone(req)
        for k in ("rhoA", "rhoB", "ux", "uy"):
            assert np.array_equal(got[k], ref[k]), (req.rid, k)
    print(f"  p50 {out['p50_latency_s']:.4f} s, p99 {out['p99_latency_s']:.4f} s", flush=True)


def test_admission_respects_budget_and_slots():
    """Budget and slot limits hold at every moment; a request larger than the
    whole budget, arriving mid-trace, is rejected and holds up nothing."""
    from paper_0807_4471_amd import serving
    banner("serving: HBM budget and slots, one request too large for the budget")
    trace = _trace()
    budget = 2 * max(serving.footprint(r) for r in trace)
    big = serving.Request(rid=len(trace), arrival=trace[3].arrival, nx=1024, ny=1024, steps=10,
                          seed=99)
    assert serving.footprint(big) > budget
    trace = trace + [big]
    live, peak_bytes, peak_n = {}, 0, 0

    def ev(kind, rid, t):
        nonlocal peak_bytes, peak_n
        if kind == "admit":
            live[rid] = serving.footprint(trace[rid])
        elif kind == "finish":
            live.pop(rid)
        peak_bytes = max(peak_bytes, sum(live.values()))
        peak_n = max(peak_n, len(live))

    out = serving.Server(hbm_budget=budget, max_slots=3, chunk_ms=0.5).run(trace, on_event=ev)
    assert out["completed"] == len(trace) - 1 and out["rejected"] == 1
    assert out["results"][big.rid].status == "rejected"
    assert peak_bytes <= budget and peak_n <= 3


def test_corrupted_request_fails_alone():
    import torch
    from paper_0807_4471_amd import serving
    banner("serving: NaN in one request")
    trace = _trace()
    victim = 4

    def corrupt(req, sim):
        # first population plane, storage row 1 (a real row with or without
        # ghost rows), column 7: read by the next step
        if req.rid == victim:
            pitch = (req.nx + 63) // 64 * 64
            dt = torch.float32 if req.storage == "f32" else torch.float16
            sim.buf.view(dt)[pitch + 7] = float("nan")

    out = serving.Server(chunk_ms=0.5).run(trace, on_admit=corrupt)
    st = {r: v.status for r, v in out["results"].items()}
    assert st[victim] == "failed"
    assert all(s == "ok" for r, s in st.items() if r != victim)
    for req in trace:
        if req.rid != victim:
            ref = _alone(req)
            assert np.array_equal(out["results"][req.rid].moments["rhoA"], ref["rhoA"]), req.rid


def test_served_results_match_oracle():
    """Every request of a short overlapping trace (FP64, FP32 and FP16
    storage; periodic and moving walls) served with continuous batching,
    against the FP64 oracle run on the same request: FP64 to 1e-12, FP32 and
    FP16 within the accumulated rounding bound of helpers.accumulated_bound
    (one-step bound summed over the steps, amplified at most as the oracle
    measures for a perturbation of the same request)."""
    from helpers import WORKLOAD, accumulated_bound, max_err, oracle_amplification, oracle_run
    from paper_0807_4471_amd import serving
    banner("serving: served results vs FP64 oracle")
    trace = serving.make_trace(9, rate=4000.0, seed=11, side=(24, 72), steps=(40, 160),
                               storages=("f64", "f32", "f16dev"))
    assert {r.storage for r in trace} == {"f64", "f32", "f16dev"}
    assert {r.boundary for r in trace} == {"periodic", "walls"}
    out = serving.Server(chunk_ms=0.3).run(trace)
    assert out["completed"] == len(trace) and out["failed"] == 0
    for req in trace:
        kw = dict(WORKLOAD, wall_u=(0.0, req.wall_u))
        _, _, ref = oracle_run(req.nx, req.ny, req.steps, seed=req.seed, boundary=req.boundary,
                               **kw)
        e = max_err(out["results"][req.rid].moments, ref)
        if req.storage == "f64":
            tol = 1e-12
        else:
            amp = oracle_amplification(req.nx, req.ny, req.steps, seed=req.seed,
                                       boundary=req.boundary, **kw)
            tol = accumulated_bound(req.storage, amp, req.steps)
        print(f"  request {req.rid} {req.nx}^2 {req.storage} {req.boundary} U={req.wall_u} "
              f"steps={req.steps}: err {e}, bound {tol:.3g}", flush=True)
        assert e["rho"] <= tol and e["u"] <= tol, (req.rid, e, tol)
