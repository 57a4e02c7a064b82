"""The seeded input generator: SplitMix64 against its published test vector,
and the initial-density recipe rho_s = mean_s (1 + amp U)."""
import os

import numpy as np

from paper_0807_4471_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed1234567.txt")


def test_splitmix64_reference_vector():
    want = [int(l) for l in open(GOLD) if l.strip() and not l.startswith("#")]
    got = inputs.splitmix64(1234567, np.arange(len(want)))
    assert [int(v) for v in got] == want


def test_counter_based_equals_sequential():
    a = inputs.splitmix64(42, np.arange(100))
    b = np.array([inputs.splitmix64(42, np.array([c]))[0] for c in range(100)])
    assert np.array_equal(a, b)


def test_random_densities_recipe():
    r = inputs.random_densities(48, 40, seed=1, mean=(0.7, 0.6), amp=0.05)
    assert r.shape == (2, 40, 48)
    assert np.all(r[0] >= 0.7 * 0.95) and np.all(r[0] < 0.7 * 1.05)
    assert np.all(r[1] >= 0.6 * 0.95) and np.all(r[1] < 0.6 * 1.05)
    assert abs(r[0].mean() - 0.7) < 0.002
    assert not np.array_equal(r[0] / 0.7, r[1] / 0.6)
    r2 = inputs.random_densities(48, 40, seed=2)
    assert not np.array_equal(r[0], r2[0])
