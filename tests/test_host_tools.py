"""Host logic without a GPU: shear observables from read-outs, the traffic
summarizer that scales counter runs by a copy calibration, and bench.py's
refusal of more than one GPU."""
import csv
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_0807_4471_amd import observables

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_apparent_viscosity_of_a_linear_profile():
    """sigma = eta * du/dy exactly on a linear profile; the rows at the walls
    are excluded by construction (central differences)."""
    ny = 40
    y = np.arange(ny)
    eta = 0.123
    g = 2.5e-4
    ux = g * (y + 0.5)
    sxy = np.full(ny, eta * g)
    e, nu = observables.apparent_viscosity(ux, sxy, rho_mean=1.4)
    assert abs(e - eta) < 1e-14 and abs(nu - eta / 1.4) < 1e-14


def test_apparent_viscosity_ignores_shear_free_rows():
    """Rows without shear carry arbitrary stress and do not enter the fit."""
    ux = np.concatenate([np.zeros(10), 1e-3 * np.arange(20), np.full(10, 19e-3)])
    g = np.zeros_like(ux)
    g[1:-1] = 0.5 * (ux[2:] - ux[:-2])
    sxy = np.where(g > 0, 0.5 * g, 7.0)
    e, _ = observables.apparent_viscosity(ux, sxy, 1.0)
    assert abs(e - 0.5) < 1e-12


def test_mean_wall_stress_sign_and_scale():
    d = {"wall_mom": np.array([[0.0, 0.0], [-3.2, 0.1]]), "wall_steps": 100}
    # the fluid receives +x momentum from the top wall: it exerts -x on the
    # wall, the returned stress is positive
    assert observables.mean_wall_stress(d, nx=16) == pytest.approx(3.2 / (16 * 100))
    with pytest.raises(ValueError):
        observables.mean_wall_stress({"wall_mom": d["wall_mom"], "wall_steps": 0}, nx=16)


def test_bulk_pressure_closed_forms():
    """Ideal part only without couplings; with couplings the terms add as
    written for a uniform state."""
    P = observables.bulk_pressure(0.7, 0.3, (0, 0), (0, 0), 0.0, 0.7, 0.7)
    assert P == pytest.approx(1.0 / 3.0)
    Ga, Gr, Gx, r0, A = (-12.55, -11.8), (11.7, 10.95), 0.58, 0.7, 0.7
    ra, rb = 0.8, 0.2
    pa, pb = A * (1 - np.exp(-ra / r0)), A * (1 - np.exp(-rb / r0))
    expect = (ra + rb) / 3 + (1 / 6) * ((Ga[0] + Gr[0]) * pa ** 2 + (Ga[1] + Gr[1]) * pb ** 2) \
        + (Gx / r0) * ra * rb / 3
    assert observables.bulk_pressure(ra, rb, Ga, Gr, Gx, r0, A) == pytest.approx(expect, rel=1e-14)


def test_droplet_jump_and_laplace_fit():
    from paper_0807_4471_amd import inputs
    rho = inputs.droplet_densities(64, 64, 12.0, 1.5, 0.06, width=0.5)
    params = dict(Ga=(0, 0), Gr=(0, 0), Gx=0.0, rho0=1.0, psi_amp=1.0)
    R, dP = observables.droplet_jump(rho[0], rho[1], params)
    assert abs(R - 12.0) < 0.3 and abs(dP) < 1e-12     # ideal: rho_A + rho_B is flat
    radii = np.array([8.0, 11.0, 14.0, 17.0])
    s, c0, r2 = observables.laplace_fit(radii, 0.12 / radii + 0.003)
    assert s == pytest.approx(0.12) and c0 == pytest.approx(0.003) and r2 == pytest.approx(1.0)
    # dissolved droplets (nan) are left out; too few points give nan
    s2, _, _ = observables.laplace_fit(list(radii) + [np.nan], list(0.12 / radii) + [np.nan])
    assert s2 == pytest.approx(0.12)
    assert np.isnan(observables.laplace_fit([8.0, np.nan], [0.1, 0.2])[0])
    flat = np.full((32, 32), 0.7)
    assert np.isnan(observables.droplet_jump(flat, flat, params)[0])


def _counters(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Value"])
        w.writeheader()
        for name, grid, val in rows:
            w.writerow({"Kernel_Name": name, "Grid_Size": grid, "Counter_Value": val})


def test_traffic_summary_scales_by_the_copy(tmp_path):
    from paper_0807_4471_amd import profsummary
    from paper_0807_4471_amd.build import kernel_source_hash
    nb = 1 << 30
    _counters(tmp_path / "cf.csv", [("copy", 1024, nb / 1024 / 2), ("small", 8, 3.0)])
    _counters(tmp_path / "cw.csv", [("copy", 1024, nb / 1024)])
    _counters(tmp_path / "f.csv", [("void k<A>(int)", 100, 10.0), ("void k<A>(int)", 100, 30.0),
                                   ("void k<B>(int)", 100, 99.0)])
    _counters(tmp_path / "w.csv", [("void k<A>(int)", 100, 5.0), ("void k<A>(int)", 100, 5.0)])
    out = tmp_path / "t.json"
    profsummary.main(["traffic", "--fetch", str(tmp_path / "f.csv"), "--write",
                      str(tmp_path / "w.csv"), "--copy-fetch", str(tmp_path / "cf.csv"),
                      "--copy-write", str(tmp_path / "cw.csv"), "--copy-bytes", str(nb),
                      "--entry", "x=k<A>@100", "-o", str(out)])
    t = json.loads(out.read_text())
    assert t["kernel_hash"] == kernel_source_hash()
    assert t["calibration"]["fetch_factor"] == pytest.approx(2.0)
    # mean fetch 20 KiB x 2 + mean write 5 KiB x 1
    assert t["per_launch_bytes"]["x"] == round(20 * 1024 * 2 + 5 * 1024)


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_kernel_hash_ignores_comments_not_code(tmp_path, monkeypatch):
    from paper_0807_4471_amd import build
    src = tmp_path / "k.hip"
    src.write_text("int f(int a) { return a + 1; } // one\n/* block\n comment */\n")
    monkeypatch.setattr(build, "KERNEL_SOURCES", [str(src)])
    h0 = build.kernel_source_hash()
    src.write_text("int f(int a)  {\n  return a + 1;   // another comment\n}\n")
    assert build.kernel_source_hash() == h0
    src.write_text("int f(int a) { return a + 2; }\n")
    assert build.kernel_source_hash() != h0
