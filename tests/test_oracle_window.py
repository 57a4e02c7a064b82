"""The windowed oracle used for sampled parity on lattices too large for the
oracle as a whole: a periodic window around a site, of half-width
3*steps + 3, gives the full lattice's result at that site bit for bit (the
oracle's arithmetic does not depend on the position), and a window one
site too narrow per step does not."""
import numpy as np
import pytest

from helpers import WORKLOAD, oracle_run, oracle_window_moments, window_half_width
from paper_0807_4471_amd import inputs


def test_window_generator_matches_full_field():
    full = inputs.random_densities(37, 23, 99, mean=(0.7, 0.65), amp=0.05)
    ys = np.array([22, 0, 1, 5])
    xs = np.array([36, 0, 3])
    w = inputs.random_densities_window(37, 23, 99, ys, xs, mean=(0.7, 0.65), amp=0.05)
    assert np.array_equal(w, full[:, ys][:, :, xs])


@pytest.mark.parametrize("steps", [1, 2])
def test_window_reproduces_full_lattice_bitwise(steps):
    nx, ny, seed = 41, 37, 5
    h = window_half_width(steps)
    assert 2 * h + 1 < min(nx, ny)       # the windows really are smaller
    sites = [(0, 0), (36, 40), (18, 20), (1, 39), (35, 2)]
    got = oracle_window_moments(nx, ny, seed, sites, steps, **WORKLOAD)
    _, _, (r, ux, uy) = oracle_run(nx, ny, steps, seed=seed, **WORKLOAD)
    ref = np.array([(r[0][y, x], r[1][y, x], ux[y, x], uy[y, x]) for y, x in sites])
    assert np.array_equal(got, ref)


def test_too_narrow_window_differs():
    """Negative control: with half-width 3*steps the velocity read-out of the
    centre already sees the window's wrap-around."""
    import helpers
    nx, ny, seed, steps = 41, 37, 5, 2
    sites = [(18, 20)]
    _, _, (r, ux, uy) = oracle_run(nx, ny, steps, seed=seed, **WORKLOAD)
    ref = np.array([(r[0][18, 20], r[1][18, 20], ux[18, 20], uy[18, 20])])
    orig = helpers.window_half_width
    try:
        helpers.window_half_width = lambda s: 3 * s
        narrow = oracle_window_moments(nx, ny, seed, sites, steps, **WORKLOAD)
    finally:
        helpers.window_half_width = orig
    assert not np.array_equal(narrow, ref)


def test_column_window_with_walls_reproduces_full_lattice_bitwise():
    """Full-height windows, periodic in x, with the moving walls: the centre
    column equals the full lattice's, wall rows included."""
    from helpers import oracle_column_moments
    nx, ny, seed, steps = 41, 12, 8, 2
    kw = dict(WORKLOAD, wall_u=(0.01, -0.04))
    cols = [0, 20, 40]
    got = oracle_column_moments(nx, ny, seed, cols, steps, boundary="walls", **kw)
    _, _, (r, ux, uy) = oracle_run(nx, ny, steps, seed=seed, boundary="walls", **kw)
    for k, x in enumerate(cols):
        ref = np.stack([r[0][:, x], r[1][:, x], ux[:, x], uy[:, x]])
        assert np.array_equal(got[k], ref), x
