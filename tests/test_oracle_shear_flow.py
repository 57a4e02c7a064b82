"""Pins of the oracle's shear-flow observables (the rheology experiment: the
response R = U_bar / U0 and the interface indicator I_AB = sum grad rho_A .
grad rho_B), against closed forms:
  * I_AB of two plane waves rho_s = rho_bar_s + a_s cos(k.r + phi_s): the
    D2Q9 gradient of exp(i k.r) is i g(k) exp(i k.r) with the real symbol
    g(k) = 3 sum_i w_i c_i sin(k.c_i), so I_AB = a_A a_B |g|^2 N cos(phi_A -
    phi_B) / 2 exactly (sums of sin^2 over whole periods);
  * U_bar of a pure sine velocity field is its amplitude;
  * a plain fluid (G = 0) under the Kolmogorov body force rho F0 sin(k y)
    relaxes to u_x = F0 / (nu k^2) sin(k y) (Navier-Stokes; lattice
    corrections O(k^2/12)), i.e. R = 1 when U0 = F0 / (nu k^2).
"""
import math

import numpy as np
import pytest

CS2 = 1.0 / 3.0
C = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
W = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4


def _state(oracle_lib, p, rho, ux=None):
    return oracle_lib.init(p, rho, ux, None)


@pytest.mark.parametrize("m,n,phi", [(1, 0, 0.0), (0, 2, 0.7), (3, 1, 2.0), (2, 5, -1.1)])
def test_iab_of_plane_waves(oracle_lib, m, n, phi):
    nx, ny = 24, 20
    p = oracle_lib.Params(nx=nx, ny=ny, Ga=(0, 0), Gr=(0, 0), Gx=0.0)
    kx, ky = 2 * math.pi * m / nx, 2 * math.pi * n / ny
    y, x = np.mgrid[0:ny, 0:nx]
    th = kx * x + ky * y
    aA, aB = 0.03, 0.05
    rho = np.stack([0.7 + aA * np.cos(th), 0.6 + aB * np.cos(th + phi)])
    f = _state(oracle_lib, p, rho)
    g = np.array([3 * sum(w * c[d] * math.sin(kx * c[0] + ky * c[1]) for w, c in zip(W, C))
                  for d in (0, 1)])
    expect = aA * aB * (g @ g) * nx * ny * math.cos(phi) / 2
    got = oracle_lib.shear_flow(p, f)["i_ab"]
    assert abs(got - expect) <= 1e-12 * max(1.0, abs(expect)) + 1e-15, (got, expect)


def test_iab_is_zero_for_uniform_fields_and_sign_of_anti_phase(oracle_lib):
    p = oracle_lib.Params(nx=16, ny=16, Ga=(0, 0), Gr=(0, 0), Gx=0.0)
    f = _state(oracle_lib, p, np.full((2, 16, 16), 0.7))
    assert oracle_lib.shear_flow(p, f)["i_ab"] == 0.0
    x = np.arange(16)
    wave = np.tile(0.02 * np.cos(2 * math.pi * x / 16), (16, 1))
    f = _state(oracle_lib, p, np.stack([0.7 + wave, 0.7 - wave]))   # interfaces: A up, B down
    assert oracle_lib.shear_flow(p, f)["i_ab"] < 0.0


def test_u_bar_of_a_sine_field(oracle_lib):
    nx, ny, U = 12, 32, 0.02
    p = oracle_lib.Params(nx=nx, ny=ny, Ga=(0, 0), Gr=(0, 0), Gx=0.0)
    y = np.arange(ny)
    ux = np.tile((U * np.sin(2 * math.pi * y / ny))[:, None], (1, nx))
    f = _state(oracle_lib, p, np.full((2, ny, nx), 0.5), ux)
    assert abs(oracle_lib.shear_flow(p, f)["u_bar"] - U) < 1e-15


@pytest.mark.parametrize("forcing", ["shift", "guo"])
@pytest.mark.parametrize("tau", [0.8, 1.0])
def test_kolmogorov_flow_response_of_a_plain_fluid(oracle_lib, tau, forcing):
    nx, ny, U0 = 4, 32, 0.01
    k = 2 * math.pi / ny
    nu = CS2 * (tau - 0.5)
    F0 = nu * k * k * U0
    p = oracle_lib.Params(nx=nx, ny=ny, tau=(tau, tau), Ga=(0, 0), Gr=(0, 0), Gx=0.0,
                          body_F0=F0, forcing=forcing)
    f = _state(oracle_lib, p, np.full((2, ny, nx), 0.5))
    oracle_lib.run(p, f, int(12 / (nu * k * k)))          # 12 viscous times
    R = oracle_lib.shear_flow(p, f)["u_bar"] / U0
    assert abs(R - 1.0) < 0.01, R
    # the response is linear in the forcing and vanishes without it
    p0 = oracle_lib.Params(nx=nx, ny=ny, tau=(tau, tau), Ga=(0, 0), Gr=(0, 0), Gx=0.0)
    f0 = _state(oracle_lib, p0, np.full((2, ny, nx), 0.5))
    oracle_lib.run(p0, f0, 200)
    assert abs(oracle_lib.shear_flow(p0, f0)["u_bar"]) < 1e-16
