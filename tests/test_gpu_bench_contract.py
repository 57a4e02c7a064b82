"""bench.py's one JSON line, in a short configuration: every field of the
contract, with the roofline and CPU-baseline objects, is present and
consistent."""
import json
import os
import subprocess
import sys

import pytest

from helpers import banner

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_line_contract():
    banner("bench.py short run, JSON contract")
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "300", "--warmup", "20",
           "--no-sweep", "--no-dram", "--no-shear", "--no-rheology", "--no-ageing",
           "--no-laplace", "--no-batch", "--no-serve", "--no-guo", "--no-small",
           "--cpu-scale", "0.01", "--repeats", "2"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1, r.stdout
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 300 and d["warmup"] == 20
    assert d["unit"] == "MLUPS" and d["higher_is_better"] is True and d["vs_baseline"] is None
    assert d["data"] == "synthetic" and "workload" in d["config"]
    # value is the throughput implied by the time per step
    assert abs(d["value"] - 512 * 512 / (d["ms_per_step"] * 1e-3) / 1e6) <= 0.01 * d["value"]
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-3
    assert abs(rf["achieved"] - 144 * 512 * 512 / (d["ms_per_step"] * 1e-3) / 1e9) \
        <= 0.01 * rf["achieved"]
    assert rf["traffic"] is None or rf["traffic"] > 0
    dw = d["device_warmup"]
    assert dw["ms"] >= 0 and "exactly" in dw["what"]
    rp = d["repeats"]
    assert rp["runs"] == 2
    assert rp["min_us_per_step"] <= rp["median_us_per_step"] <= rp["max_us_per_step"]
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["unit"] == "MLUPS" and cb["cores"] >= 1
    assert cb["value"] > 0 and f"on {cb['cores']} threads" in cb["sample"]
    # the oracle at three sizes, single-threaded and on all the process's threads
    runs = cb["runs"]
    assert sorted({r["nx"] for r in runs}) == [64, 512, 1024]
    for nx in (64, 512, 1024):
        th = sorted(r["threads"] for r in runs if r["nx"] == nx)
        assert th[0] == 1 and th[-1] == cb["cores"]
    assert all(r["steps"] >= 1 and r["mlups"] > 0 for r in runs)
    head = [r for r in runs if r["nx"] == 512 and r["threads"] == cb["cores"]]
    assert head and head[-1]["mlups"] == cb["value"]
