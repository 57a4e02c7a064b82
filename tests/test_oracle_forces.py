"""Pins of the oracle's pseudo-potential forces (the FORCE equations).

Each test is a consequence of the force definition that does not re-type the
oracle's sums:
  * a point source of Psi (or rho) exposes every one of the 24 offsets with
    its own weight and direction;
  * for a long-wave Fourier mode the force expands as
        F = -c_s^2 G_s1 Psi grad Psi + (c_s^4 / 2) G_s2 Psi grad(lap Psi) + ...
    with the paper's effective couplings G_s1 = G^a + G^r and
    G_s2 = G^a + (12/7) G^r; positive couplings must repel;
  * the repulsion stencil is isotropic to 8th order, so its Fourier symbol
    depends on |k| only up to O(k^9);
  * the interaction forces sum to zero over a periodic lattice.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from test_oracle_stencil import exact_d2q9_weights, exact_repulsion_weights

CS2 = 1.0 / 3.0


def P(oracle_lib, **kw):
    base = dict(nx=11, ny=9, Ga=(0.0, 0.0), Gr=(0.0, 0.0), Gx=0.0, rho0=0.7, psi_amp=0.7)
    base.update(kw)
    return oracle_lib.Params(**base)


def test_psi_special_values(oracle_lib):
    p = P(oracle_lib, rho0=0.6, psi_amp=0.9)
    assert oracle_lib.psi(p, 0.0) == 0.0
    assert abs(oracle_lib.psi(p, 0.6) - 0.9 * (1.0 - math.exp(-1.0))) < 1e-16
    assert abs(oracle_lib.psi(p, 60.0) - 0.9) < 1e-15
    h = 1e-7
    slope = oracle_lib.psi(p, h) / h
    assert abs(slope - 0.9 / 0.6) < 1e-6          # Psi'(0) = A / rho0
    # monotone and concave
    r = np.linspace(0.0, 3.0, 31)
    v = np.array([oracle_lib.psi(p, x) for x in r])
    assert np.all(np.diff(v) > 0) and np.all(np.diff(v, 2) < 0)


def test_feq_moments(oracle_lib):
    cx, cy, w = oracle_lib.d2q9()
    for rho, ux, uy in [(1.0, 0.0, 0.0), (0.7, 0.05, -0.03), (1.3, -0.1, 0.08)]:
        f = oracle_lib.feq(rho, ux, uy)
        assert abs(f.sum() - rho) < 1e-15
        assert abs((f * cx).sum() - rho * ux) < 1e-16
        assert abs((f * cy).sum() - rho * uy) < 1e-16
        assert abs((f * cx * cx).sum() - (rho * CS2 + rho * ux * ux)) < 1e-15
        assert abs((f * cy * cy).sum() - (rho * CS2 + rho * uy * uy)) < 1e-15
        assert abs((f * cx * cy).sum() - rho * ux * uy) < 1e-16


@pytest.mark.parametrize("Ga,Gr", [(1.0, 0.0), (0.0, 1.0), (-12.55, 11.70)])
def test_point_source_psi(oracle_lib, Ga, Gr):
    """F_s(x0 - e) = -(G^a w(e) + G^r p(e)) Psi_bar delta e for each offset e."""
    nx, ny = 11, 9
    p = P(oracle_lib, nx=nx, ny=ny, Ga=(Ga, 0.0), Gr=(Gr, 0.0))
    pw, _ = exact_repulsion_weights()
    _, ww = exact_d2q9_weights()
    pbar, delta = 0.4, 0.125
    psi = np.full((2, ny, nx), pbar)
    x0, y0 = 5, 4
    psi[0, y0, x0] += delta
    rho = np.full((2, ny, nx), 0.7)
    F = oracle_lib.forces(p, psi, rho)
    exp = np.zeros((2, ny, nx))
    for ex in range(-2, 3):
        for ey in range(-2, 3):
            e2 = ex * ex + ey * ey
            if e2 == 0:
                continue
            K = Ga * float(ww.get(e2, Fraction(0))) + Gr * float(pw[e2])
            exp[0, (y0 - ey) % ny, (x0 - ex) % nx] = -K * pbar * delta * ex
            exp[1, (y0 - ey) % ny, (x0 - ex) % nx] = -K * pbar * delta * ey
    np.testing.assert_allclose(F[0], exp, rtol=0, atol=1e-15)
    assert np.all(F[1] == 0.0)          # species B is uniform and G^X = 0


def test_point_source_rho_cross(oracle_lib):
    """F^X uses the other species' density: a bump in rho_B pushes A away
    (G_AB > 0 repels) and leaves B's own cross force at zero."""
    nx, ny = 11, 9
    Gx, rho0 = 0.58, 0.7
    p = P(oracle_lib, nx=nx, ny=ny, Gx=Gx, rho0=rho0)
    _, ww = exact_d2q9_weights()
    rA, rB, delta = 0.6, 0.8, 0.25
    rho = np.empty((2, ny, nx))
    rho[0] = rA
    rho[1] = rB
    x0, y0 = 3, 6
    rho[1, y0, x0] += delta
    psi = np.full((2, ny, nx), 0.3)
    F = oracle_lib.forces(p, psi, rho)
    exp = np.zeros((2, ny, nx))
    for ex in (-1, 0, 1):
        for ey in (-1, 0, 1):
            e2 = ex * ex + ey * ey
            if e2 == 0:
                continue
            k = -(Gx / rho0) * rA * float(ww[e2]) * delta
            exp[0, (y0 - ey) % ny, (x0 - ex) % nx] = k * ex
            exp[1, (y0 - ey) % ny, (x0 - ex) % nx] = k * ey
    np.testing.assert_allclose(F[0], exp, rtol=0, atol=1e-15)
    # repulsion: the A force at the site left of the bump points left (away)
    assert F[0, 0, y0, x0 - 1] < 0.0
    assert np.all(np.abs(F[1]) < 1e-15)


def _mode_symbol(oracle_lib, Ga, Gr, L, m, n, amp=1e-3):
    """S(k) from F(x) = eps Psi(x) sin(k.x) S(k) for Psi = Psi_bar + eps cos(k.x)."""
    p = P(oracle_lib, nx=L, ny=L, Ga=(Ga, Ga), Gr=(Gr, Gr))
    y, x = np.mgrid[0:L, 0:L].astype(float)
    kx, ky = 2 * np.pi * m / L, 2 * np.pi * n / L
    ph = kx * x + ky * y
    psi = np.empty((2, L, L))
    psi[:] = 0.45 + amp * np.cos(ph)
    rho = np.full((2, L, L), 0.7)
    F = oracle_lib.forces(p, psi, rho)
    den = amp * psi[0] * np.sin(ph)
    sel = np.abs(np.sin(ph)) > 0.5
    Sx = (F[0, 0][sel] / den[sel])
    Sy = (F[0, 1][sel] / den[sel])
    assert np.ptp(Sx) < 1e-9 * max(1.0, abs(Sx).max())   # single-mode closed form
    return np.array([Sx.mean(), Sy.mean()]), np.array([kx, ky])


@pytest.mark.parametrize("Ga,Gr", [(1.0, 0.0), (0.0, 1.0), (-12.55, 11.70), (-11.80, 10.95)])
def test_long_wave_expansion_effective_couplings(oracle_lib, Ga, Gr):
    """S(k)/|k| = c_s^2 G1 - (c_s^4/2) G2 k^2 + O(k^4), G1 = G^a + G^r,
    G2 = G^a + (12/7) G^r (the paper's effective couplings)."""
    G1 = Ga + Gr
    G2 = Ga + 12.0 / 7.0 * Gr
    L = 512
    a = []
    ks = []
    for m in (1, 2):
        S, k = _mode_symbol(oracle_lib, Ga, Gr, L, m, 0)
        kk = k[0]
        assert abs(S[1]) < 1e-12 * abs(S[0]) + 1e-18
        ks.append(kk)
        a.append((S[0] / kk - CS2 * G1) / kk ** 2)
        assert abs(S[0] / kk - CS2 * G1) < 0.01 * max(abs(G1), abs(G2)) + 1e-12
    # Richardson extrapolation of the k^2 coefficient
    c2 = (4 * a[0] - a[1]) / 3
    assert abs(c2 - (-CS2 * CS2 / 2 * G2)) < 1e-5 * max(1.0, abs(G2)), (c2, G2)


def test_repulsive_sign(oracle_lib):
    """Positive couplings repel: for G^r > 0 the force points down the Psi
    gradient (away from the denser region)."""
    S, k = _mode_symbol(oracle_lib, 0.0, 1.0, 64, 1, 0)
    assert S[0] > 0.0
    S, k = _mode_symbol(oracle_lib, -1.0, 0.0, 64, 1, 0)
    assert S[0] < 0.0


def test_repulsion_stencil_isotropy(oracle_lib):
    """8th-order isotropy: |S(k)| of the p stencil is the same for k along
    (5,0) and (3,4) to O(k^9); the 4th-order D2Q9 stencil is not."""
    L = 64
    Sa, ka = _mode_symbol(oracle_lib, 0.0, 1.0, L, 5, 0, amp=1e-2)
    Sb, kb = _mode_symbol(oracle_lib, 0.0, 1.0, L, 3, 4, amp=1e-2)
    assert abs(np.linalg.norm(ka) - np.linalg.norm(kb)) < 1e-14
    rel_p = abs(np.linalg.norm(Sa) - np.linalg.norm(Sb)) / np.linalg.norm(Sa)
    cross = abs(Sb[0] * kb[1] - Sb[1] * kb[0]) / (np.linalg.norm(Sb) * np.linalg.norm(kb))
    Wa, _ = _mode_symbol(oracle_lib, 1.0, 0.0, L, 5, 0, amp=1e-2)
    Wb, _ = _mode_symbol(oracle_lib, 1.0, 0.0, L, 3, 4, amp=1e-2)
    rel_w = abs(np.linalg.norm(Wa) - np.linalg.norm(Wb)) / np.linalg.norm(Wa)
    assert rel_p < 1e-7 and cross < 1e-7, (rel_p, cross)
    assert rel_w > 1e-4, rel_w
    assert rel_w > 1000 * rel_p


def test_zero_net_force(oracle_lib):
    """Sum_x F^Psi_s = 0 per species; Sum_x (F^X_A + F^X_B) = 0 over both."""
    rng = np.random.default_rng(7)
    nx, ny = 13, 10
    psi = 0.4 + 0.1 * rng.random((2, ny, nx))
    rho = 0.7 + 0.2 * rng.random((2, ny, nx))
    p = P(oracle_lib, nx=nx, ny=ny, Ga=(-12.55, -11.80), Gr=(11.70, 10.95))
    F = oracle_lib.forces(p, psi, rho)
    scale = np.abs(F).sum()
    assert np.all(np.abs(F.sum(axis=(2, 3))) < 1e-13 * scale)
    p = P(oracle_lib, nx=nx, ny=ny, Gx=0.58)
    F = oracle_lib.forces(p, psi, rho)
    scale = np.abs(F).sum()
    per = F.sum(axis=(2, 3))
    assert np.all(np.abs(per.sum(axis=0)) < 1e-13 * scale)
    assert np.abs(per).max() > 1e-6 * scale      # each species alone does not vanish


def test_uniform_fields_give_no_force(oracle_lib):
    p = P(oracle_lib, Ga=(-12.55, -11.80), Gr=(11.70, 10.95), Gx=0.58)
    psi = np.full((2, 9, 11), 0.44248)
    rho = np.full((2, 9, 11), 0.7)
    F = oracle_lib.forces(p, psi, rho)
    assert np.abs(F).max() < 1e-15
