"""The uneven batch workload's 128x128 instances, advanced together for 500
steps in one batch (both execution modes): the instances the kernels flag
with non-positive densities must be exactly those the FP64 oracle finds
(tests/golden/batch_mix_divergence.json, written from the oracle alone), and
in FP64 every member must match the oracle's densities."""
import json
import os

import numpy as np
import pytest

from helpers import WORKLOAD, accumulated_bound, banner, oracle_amplification

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                    "batch_mix_divergence.json")


def _batch(storage, mode):
    from paper_0807_4471_amd import inputs, sclbm
    with open(GOLD) as fh:
        gold = json.load(fh)
    mix = inputs.batch_mix()
    rows = gold["instances"]
    sims = []
    for r in rows:
        m = mix[r["instance"]]
        s = sclbm.Simulation(m["nx"], m["ny"], storage=storage,
                             **{**WORKLOAD, "rho0": m["rho0"], "Gx": m["Gx"], "tau": m["tau"]})
        s.init_random(m["seed"])
        sims.append(s)
    b = sclbm.Batch(sims, mode=mode)
    b.step(gold["steps"])
    b.status()
    b.close()
    return rows, mix, sims, gold["steps"]


@pytest.mark.parametrize("mode", ["stepwise", "persistent"])
def test_f64_batch_flags_the_oracle_instances_and_matches_it(mode):
    banner(f"f64 {mode} batch of the 13 128^2 mix instances, 500 steps, vs oracle")
    rows, mix, sims, steps = _batch("f64", mode)
    for r, s in zip(rows, sims):
        bad = s.diagnostics()["bad_sites"]
        m = mix[r["instance"]]
        amp, ref = oracle_amplification(
            m["nx"], m["ny"], steps, seed=m["seed"], with_moments=True,
            **{**WORKLOAD, "rho0": m["rho0"], "Gx": m["Gx"], "tau": m["tau"]})
        tol = accumulated_bound("f64", amp, steps)
        got = s.moments()
        err = max(np.abs(got["rhoA"] - ref[0][0]).max(), np.abs(got["rhoB"] - ref[0][1]).max())
        print(f"  instance {r['instance']}: bad {bad} (oracle {r['bad_sites']}), "
              f"max|drho| {err:.3g}, bound {tol:.3g} (growth {amp[-1]:.3g})", flush=True)
        assert bad == r["bad_sites"], r
        assert err <= tol, (r["instance"], err, tol)


@pytest.mark.parametrize("mode", ["stepwise", "persistent"])
def test_f32_batch_flags_the_oracle_instances(mode):
    """The benchmark's storage: FP32 flags exactly the instances the oracle
    flags.  Site counts may differ by a few where FP32 rounding tips a site
    near rho = 0 either way: within 1% + 3 sites."""
    banner(f"f32 {mode} batch of the 13 128^2 mix instances, 500 steps")
    rows, _, sims, _ = _batch("f32", mode)
    got = {}
    for r, s in zip(rows, sims):
        bad = s.diagnostics()["bad_sites"]
        got[r["instance"]] = bad
        print(f"  instance {r['instance']}: bad {bad} (oracle {r['bad_sites']})", flush=True)
        assert abs(bad - r["bad_sites"]) <= 0.01 * r["bad_sites"] + 3, (bad, r)
    assert {i for i, b in got.items() if b > 0} == {r["instance"] for r in rows
                                                    if r["bad_sites"] > 0}
