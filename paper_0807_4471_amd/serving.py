"""Continuous-batching server for lattice Boltzmann solve requests.

Requests (lattice size, steps, storage, boundary, seed, physical parameters)
arrive over time.  The server admits them in arrival order as soon as their
device state fits the HBM budget and a slot is free, keeps every admitted
state on the device, and advances all active instances of a storage type
together in batch calls (``sclbm.Batch``, tuned tiles and execution mode)
of about `chunk_ms` each.  Within a chunk every request advances the same
number of steps, or (work-fair slicing) small lattices take up to a few
times more.  New arrivals join at the next chunk; an instance that reaches its step
count inside a chunk drops out of that call.  Finished requests are retired:
their FP64 diagnostics are checked (a non-finite state marks that request
failed and affects no other), their moments are read back to the host, their
buffers are freed.

Each request's result is bitwise the result of running it alone, because a
batch launch performs exactly the per-site arithmetic of a single-instance
step (tested).

The clock is the host wall clock from the start of `run`; a request's
latency is its completion time minus its arrival time.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

WORKLOAD = dict(Ga=(-12.55, -11.80), Gr=(11.70, 10.95), Gx=0.58, rho0=0.70)


@dataclass
class Request:
    rid: int
    arrival: float            # seconds from the start of the trace
    nx: int
    ny: int
    steps: int
    storage: str = "f32"      # "f32", "f16sr" (FP16 deviations rounded
                              # stochastically), "f16dev" or "f64"
    boundary: str = "periodic"
    wall_u: float = 0.0       # top-wall speed for boundary == "walls"
    seed: int = 0
    params: dict = field(default_factory=dict)

    @property
    def sites(self) -> int:
        return self.nx * self.ny

    @property
    def work(self) -> int:
        return self.nx * self.ny * self.steps


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float
    status: str               # "ok", "failed" (non-finite state) or "rejected"
                              # (footprint above the server's HBM budget)
    moments: dict | None
    diag: dict | None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def make_trace(n: int, rate: float, seed: int = 4242, side=(64, 1024), steps=(1000, 100000),
               storages=("f32", "f16sr"), walls_fraction=0.5,
               wall_speeds=(0.01, 0.05, 0.1)) -> list[Request]:
    """Poisson arrivals at `rate` per second; sizes and step counts
    log-uniform; storage and boundary drawn uniformly; per-request seeds
    10000 + id.  FP16 requests store deviations rounded stochastically:
    round-to-nearest is biased in steady wall-driven flow, which half of the
    requests are."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        s = int(round(math.exp(rng.uniform(math.log(side[0]), math.log(side[1])))))
        st = int(round(math.exp(rng.uniform(math.log(steps[0]), math.log(steps[1])))))
        walls = rng.uniform() < walls_fraction
        out.append(Request(rid=i, arrival=t, nx=s, ny=s, steps=st,
                           storage=storages[int(rng.integers(len(storages)))],
                           boundary="walls" if walls else "periodic",
                           wall_u=float(rng.choice(wall_speeds)) if walls else 0.0,
                           seed=10000 + i))
    return out


def _new_sim(req: Request, device):
    from . import sclbm
    kw = dict(WORKLOAD)
    kw.update(req.params)
    sim = sclbm.Simulation(req.nx, req.ny, device=device, storage=req.storage,
                           boundary=req.boundary, wall_u=(0.0, req.wall_u), rho_ref=(0.7, 0.7),
                           **kw)
    sim.init_random(req.seed)
    return sim


def footprint(req: Request) -> int:
    from . import sclbm
    return sclbm.state_bytes(sclbm.make_desc(req.nx, req.ny, storage=req.storage,
                                             boundary=req.boundary))


class Server:
    """Continuous batching over one GPU.

    hbm_budget: bytes of instance state allowed on the device at once.
    max_slots:  instances in flight at once.
    chunk_ms:   target duration of one batch call (bounds admission delay).
    slicing:    "steps" (default): every active request advances the same
                number of steps per chunk; "work": every active request gets
                an equal share of the chunk's lattice updates, between the
                step-fair count and WORK_BOOST times it (small lattices take
                more steps, so short requests finish sooner; the extra steps
                of tiny lattices are launch-bound, which costs throughput).
    """

    WORK_BOOST = 4

    def __init__(self, hbm_budget: int = 64 << 30, max_slots: int = 256, chunk_ms: float = 20.0,
                 device: str = "cuda", keep_moments: bool = True, tiling: str = "auto",
                 slicing: str = "steps"):
        if slicing not in ("work", "steps"):
            raise ValueError("slicing must be 'work' or 'steps'")
        if int(hbm_budget) <= 0:
            raise ValueError("hbm_budget must be > 0 bytes")
        if int(max_slots) < 1:
            raise ValueError("max_slots must be >= 1")
        if not float(chunk_ms) > 0.0:
            raise ValueError("chunk_ms must be > 0")
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.chunk_ms = float(chunk_ms)
        self.device = device
        self.keep_moments = keep_moments
        self.tiling = tiling
        self.slicing = slicing
        self.rate_lups = 2.0e10  # running estimate of batch throughput (LUP/s)

    def _slice(self, active, order, total_sites):
        """Steps of each request in `order` for the next chunk."""
        budget = self.rate_lups * self.chunk_ms * 1e-3      # lattice updates per chunk
        chunk = max(1, int(budget / max(1, total_sites)))
        if self.slicing == "steps":
            return [min(active[r][2], chunk) for r in order]
        share = budget / max(1, len(active))
        return [min(active[r][2], self.WORK_BOOST * chunk,
                    max(chunk, int(share / active[r][0].sites))) for r in order]


    def run(self, trace: list[Request], on_event=None, on_admit=None) -> dict:
        """Serve the trace in real time; returns results and metrics.
        on_event(kind, rid, t) is told of admissions and completions;
        on_admit(req, sim) may inspect (or, in tests, corrupt) a new state."""
        import torch
        from . import sclbm
        pending = sorted(trace, key=lambda r: r.arrival)
        active = {}          # rid -> [req, sim, remaining, admitted_at]
        results = {}
        used = 0
        pi = 0
        t0 = time.perf_counter()
        busy = 0.0
        plans = {}           # storage -> (frozenset(rids), Batch)
        nchunks = nplans = 0
        active_sum = 0
        while pi < len(pending) or active:
            now = time.perf_counter() - t0
            # admission, FIFO
            while pi < len(pending) and pending[pi].arrival <= now:
                req = pending[pi]
                need = footprint(req)
                if need > self.budget:
                    # can never fit, even alone: refuse it now instead of
                    # holding the queue (and everything behind it) forever
                    results[req.rid] = Result(req.rid, req.arrival, now, now, "rejected",
                                              None, None)
                    pi += 1
                    if on_event:
                        on_event("reject", req.rid, now)
                    continue
                if len(active) >= self.max_slots or used + need > self.budget:
                    break
                sim = _new_sim(req, self.device)
                if on_admit:
                    on_admit(req, sim)
                active[req.rid] = [req, sim, req.steps, now]
                used += need
                pi += 1
                if on_event:
                    on_event("admit", req.rid, now)
            if not active:
                if pi >= len(pending):
                    break  # everything left was rejected
                # idle until the next arrival
                wait = pending[pi].arrival - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.05))
                continue
            # one chunk per storage group
            groups = {}
            for rid, (req, sim, rem, _) in active.items():
                groups.setdefault(req.storage, []).append(rid)
            total_sites = sum(active[r][0].sites for r in active)
            tc = time.perf_counter()
            work = 0
            for storage, rids in sorted(groups.items()):
                rids = sorted(rids)
                keyset = frozenset(rids)
                if storage not in plans or plans[storage][0] != keyset:
                    if storage in plans:
                        plans[storage][1].close()
                    sims = [active[r][1] for r in rids]
                    plans[storage] = (keyset, sclbm.Batch(sims, "auto" if self.tiling == "auto"
                                                          else None), rids)
                    nplans += 1
                _, batch, order = plans[storage]
                steps = self._slice(active, order, total_sites)
                batch.step(steps)
                for r, s in zip(order, steps):
                    active[r][2] -= s
                    work += active[r][0].sites * s
            torch.cuda.synchronize()
            dt = time.perf_counter() - tc
            busy += dt
            nchunks += 1
            active_sum += len(active)
            if dt > 0 and work > 0:
                self.rate_lups = 0.7 * self.rate_lups + 0.3 * (work / dt)
            # retire finished requests
            done = [r for r, v in active.items() if v[2] == 0]
            for rid in done:
                req, sim, _, adm = active.pop(rid)
                d = sim.diagnostics()
                status = "ok" if d["bad_sites"] == 0 else "failed"
                mom = sim.moments() if self.keep_moments else None
                fin = time.perf_counter() - t0
                results[rid] = Result(rid, req.arrival, adm, fin, status, mom, d)
                used -= footprint(req)
                sim.close()
                if on_event:
                    on_event("finish", rid, fin)
            if done:
                for st in list(plans):
                    if plans[st][0] & set(done):
                        plans[st][1].close()
                        del plans[st]
        makespan = time.perf_counter() - t0
        for st in plans:
            plans[st][1].close()
        out = summarize(trace, results, makespan, busy)
        out.update({"chunks": nchunks, "plans_built": nplans,
                    "mean_active": active_sum / max(1, nchunks)})
        return out


def serve_sequential_f64(trace: list[Request], device="cuda", keep_moments=False,
                         on_event=None) -> dict:
    """Baseline: the same trace served one request at a time, in arrival
    order, each on the single-instance FP64 path (sclbm_step).  on_event as
    for Server.run."""
    import torch
    from . import sclbm
    pending = sorted(trace, key=lambda r: r.arrival)
    results = {}
    t0 = time.perf_counter()
    busy = 0.0
    for req in pending:
        now = time.perf_counter() - t0
        if req.arrival > now:
            time.sleep(req.arrival - now)
        adm = time.perf_counter() - t0
        if on_event:
            on_event("admit", req.rid, adm)
        r64 = Request(**{**req.__dict__, "storage": "f64"})
        tc = time.perf_counter()
        sim = _new_sim(r64, device)
        sim.step(req.steps)
        d = sim.diagnostics()
        torch.cuda.synchronize()
        busy += time.perf_counter() - tc
        mom = sim.moments() if keep_moments else None
        fin = time.perf_counter() - t0
        results[req.rid] = Result(req.rid, req.arrival, adm, fin,
                                  "ok" if d["bad_sites"] == 0 else "failed", mom, d)
        sim.close()
        if on_event:
            on_event("finish", req.rid, fin)
    return summarize(trace, results, time.perf_counter() - t0, busy)


def summarize_public(s: dict) -> dict:
    """The metrics of `summarize` without the per-request results."""
    return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in s.items()
            if k != "results"}


def summarize(trace, results: dict, makespan: float, busy: float) -> dict:
    """Latency percentiles and throughput over the requests that ran (ok or
    failed); rejected requests are counted apart."""
    ran = [r for r in trace if r.rid in results and results[r.rid].status != "rejected"]
    lat = np.array([results[r.rid].latency for r in ran])
    work = sum(r.work for r in ran)
    failed = sum(1 for r in results.values() if r.status == "failed")
    rejected = sum(1 for r in results.values() if r.status == "rejected")
    return {
        "requests": len(trace), "completed": len(ran), "failed": failed, "rejected": rejected,
        "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else None,
        "mean_latency_s": float(lat.mean()) if len(lat) else None,
        "makespan_s": makespan, "busy_s": busy,
        "aggregate_mlups": work / makespan / 1e6 if makespan > 0 else None,
        "busy_mlups": work / busy / 1e6 if busy > 0 else None,
        "results": results,
    }
