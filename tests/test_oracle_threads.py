"""The oracle's row loops run in parallel (OpenMP).  Every site computes and
writes only its own values, and the wall-momentum sums stay in site order,
so 1 thread and several threads must agree bit for bit: populations,
wall momentum and every read-out."""
import numpy as np
import pytest

import oracle
from paper_0807_4471_amd import inputs

WORKLOAD = dict(Ga=(-12.55, -11.80), Gr=(11.70, 10.95), Gx=0.58, rho0=0.70)

CASES = {
    "periodic": dict(nx=37, ny=29),
    "walls": dict(nx=33, ny=21, walls=True, wall_u=(-0.02, 0.08)),
    "body_force_guo": dict(nx=24, ny=40, body_F0=1e-5, forcing="guo", tau=(0.8, 1.3)),
}


def _run(case, threads):
    oracle.set_threads(threads)
    p = oracle.Params(**{**WORKLOAD, **CASES[case]})
    f = oracle.init(p, inputs.random_densities(p.nx, p.ny, 5))
    wm = np.zeros((2, 2))
    oracle.run(p, f, 40, wm)
    rho, ux, uy = oracle.moments(p, f)
    tot = oracle.totals(p, f)
    prof = oracle.row_profiles(p, f)
    sf = oracle.shear_flow(p, f)
    return f, wm, rho, ux, uy, tot, prof, sf


@pytest.mark.parametrize("case", list(CASES))
def test_thread_count_does_not_change_results(case):
    try:
        one = _run(case, 1)
        many = _run(case, 4)
    finally:
        oracle.set_threads(0)
    for a, b in zip(one[:5], many[:5]):
        assert np.array_equal(a, b)
    assert all(np.array_equal(one[5][k], many[5][k]) for k in one[5])
    assert np.array_equal(one[6][0], many[6][0]) and np.array_equal(one[6][1], many[6][1])
    assert one[7] == many[7]


def test_set_threads_reports_what_it_set():
    try:
        assert oracle.set_threads(3) == 3 and oracle.threads() == 3
        assert oracle.set_threads(0) >= 1
    finally:
        oracle.set_threads(0)
