"""Brute force on tiny lattices: a whole-array numpy evaluation of the step,
written from the definitions, against the oracle's site loops.

The evaluator shares nothing with the oracle but the readings of the paper
(leading minus sign of the forces, velocity-shift forcing, second-order
equilibrium, half-way bounce-back with mirrored ghost rows).  It differs
from the oracle wherever a mistake could hide:
  * forces are sums over all 24 offsets e of K(|e|^2) e Psi(x + e) with the
    couplings folded into one kernel K = G^a w + G^r p, built from weights
    solved exactly from the paper's constraints (not the oracle's tables);
    the oracle also sums every offset on its own (no pairing of e with -e),
    but keeps separate sums for the attractive, repulsive and cross terms
    and multiplies by the couplings afterwards, in a different order;
  * neighbours come from np.roll / np.pad of whole fields (the oracle wraps
    indices per site);
  * streaming pushes whole planes with np.roll (the oracle loops over
    destination sites);
  * bounce-back is applied to the populations that a roll carried across a
    wall (the oracle tests each destination row).
So a wrong offset, a transposed index, a lost wrap, a sign or a dropped term
in either one shows up as a difference far above rounding.
"""
import numpy as np
import pytest

from paper_0807_4471_amd import inputs
from test_oracle_stencil import exact_d2q9_weights, exact_repulsion_weights

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]
CS2 = 1.0 / 3.0


def _weights():
    w0, w = exact_d2q9_weights()
    p, _ = exact_repulsion_weights()
    W = np.array([float(w0)] + [float(w[1])] * 4 + [float(w[2])] * 4)
    wsh = {k: float(v) for k, v in w.items()}
    psh = {k: float(v) for k, v in p.items()}
    return W, wsh, psh


def _offsets():
    return [(ex, ey) for ey in range(-2, 3) for ex in range(-2, 3) if ex or ey]


def _shift(field, ex, ey, walls):
    """field(x + e) for every x: periodic in x; in y periodic, or mirrored
    about the wall planes y = -1/2 and y = ny - 1/2."""
    if not walls:
        return np.roll(field, (-ey, -ex), axis=(0, 1))
    ny = field.shape[0]
    padded = np.pad(field, ((2, 2), (0, 0)), mode="symmetric")
    rows = padded[2 + ey: 2 + ey + ny]
    return np.roll(rows, -ex, axis=1)


def feq_all(W, rho, ux, uy):
    cu = CX[:, None, None] * ux + CY[:, None, None] * uy
    uu = ux * ux + uy * uy
    return W[:, None, None] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu)


def forces(f, prm):
    """Moments and forces of the state f[s, i, y, x]: rho[s], jx[s], jy[s],
    F[s, component] (interaction plus body force)."""
    W, wsh, psh = _weights()
    walls = prm["walls"]
    ny, nx = f.shape[2:]
    rho = f.sum(axis=1)
    jx = np.tensordot(CX, f, axes=([0], [1]))
    jy = np.tensordot(CY, f, axes=([0], [1]))
    psi = prm["A"] * (1.0 - np.exp(-rho / prm["rho0"]))
    F = np.zeros((2, 2, ny, nx))
    for s in range(2):
        o = 1 - s
        for ex, ey in _offsets():
            d2 = ex * ex + ey * ey
            K = prm["Ga"][s] * wsh.get(d2, 0.0) + prm["Gr"][s] * psh[d2]
            nb = _shift(psi[s], ex, ey, walls)
            F[s, 0] -= psi[s] * K * ex * nb
            F[s, 1] -= psi[s] * K * ey * nb
            if d2 <= 2:
                nr = _shift(rho[o], ex, ey, walls)
                X = prm["Gx"] / prm["rho0"] * wsh[d2]
                F[s, 0] -= rho[s] * X * ex * nr
                F[s, 1] -= rho[s] * X * ey * nr
        if prm["F0"]:
            y = np.arange(ny)[:, None]
            F[s, 0] += rho[s] * prm["F0"] * np.sin(2.0 * np.pi * y / ny)
    return rho, jx, jy, F


def step(f, prm):
    """One step of f[s, i, y, x] (post-stream populations at t) -> t + 1."""
    W, _, _ = _weights()
    walls = prm["walls"]
    ny, nx = f.shape[2:]
    rho, jx, jy, F = forces(f, prm)
    tau = prm["tau"]
    guo = prm.get("forcing", "shift") == "guo"
    if guo:   # barycentric velocity with half the force
        rt = rho[0] + rho[1]
        upx = (jx[0] + jx[1] + 0.5 * (F[0, 0] + F[1, 0])) / rt
        upy = (jy[0] + jy[1] + 0.5 * (F[0, 1] + F[1, 1])) / rt
    else:     # Shan-Chen common velocity weighted by rho_s / tau_s
        den = rho[0] / tau[0] + rho[1] / tau[1]
        upx = (jx[0] / tau[0] + jx[1] / tau[1]) / den
        upy = (jy[0] / tau[0] + jy[1] / tau[1]) / den
    out = np.zeros_like(f)
    for s in range(2):
        if guo:
            ueqx, ueqy = upx, upy
        else:
            ueqx = upx + tau[s] * F[s, 0] / rho[s]
            ueqy = upy + tau[s] * F[s, 1] / rho[s]
        fs = f[s] - (f[s] - feq_all(W, rho[s], ueqx, ueqy)) / tau[s]
        if guo:   # Guo's source: (1 - 1/(2 tau)) w_i [(c_i - u)/c_s^2 + (c_i.u) c_i / c_s^4] . F
            cu = CX[:, None, None] * upx + CY[:, None, None] * upy
            cf = CX[:, None, None] * F[s, 0] + CY[:, None, None] * F[s, 1]
            uf = upx * F[s, 0] + upy * F[s, 1]
            fs = fs + (1 - 0.5 / tau[s]) * W[:, None, None] * ((cf - uf) / CS2 + cu * cf / CS2 ** 2)
        for i in range(9):
            moved = np.roll(fs[i], (CY[i], CX[i]), axis=(0, 1))
            if walls and CY[i] != 0:
                # rows that the roll carried across a wall hold reflected
                # populations instead: f_opp(x) = f*_i(x) - 2 w_i rho (c_i.u_w)/c_s^2
                src = 0 if CY[i] > 0 else ny - 1       # wrapped-in destination row
                y_from = ny - 1 if CY[i] > 0 else 0    # the node that emitted it
                uw = prm["wall_u"][1] if CY[i] > 0 else prm["wall_u"][0]
                moved[src] = 0.0
                back = fs[i][y_from] - 2.0 * W[i] * rho[s][y_from] * (CX[i] * uw) / CS2
                out[s, OPP[i], y_from] += back
            out[s, i] += moved
    return out


def _case(nx, ny, walls, seed, F0=0.0, tau=(0.8, 1.3), wall_u=(0.0, 0.0), forcing="shift"):
    import oracle
    prm = dict(walls=walls, tau=tau, Ga=(-12.55, -11.80), Gr=(11.70, 10.95), Gx=0.58,
               rho0=0.70, A=0.70, F0=F0, wall_u=wall_u, forcing=forcing)
    p = oracle.Params(nx=nx, ny=ny, walls=walls, tau=tau, wall_u=wall_u, body_F0=F0,
                      forcing=forcing)
    rho = inputs.random_densities(nx, ny, seed, amp=0.2)
    rng = np.random.default_rng(seed)
    ux = 0.05 * rng.standard_normal((ny, nx))
    uy = 0.05 * rng.standard_normal((ny, nx))
    f0 = oracle.init(p, rho, ux, uy)
    return oracle, p, prm, f0


@pytest.mark.parametrize("forcing", ["shift", "guo"])
@pytest.mark.parametrize("nx,ny", [(8, 8), (9, 7)])
@pytest.mark.parametrize("walls", [False, True])
def test_steps_match_brute_force(oracle_lib, nx, ny, walls, forcing):
    oracle, p, prm, f0 = _case(nx, ny, walls, seed=nx * 10 + ny,
                               wall_u=(0.02, -0.05) if walls else (0.0, 0.0), forcing=forcing)
    f_or = f0.copy()
    f_bf = f0.copy()
    for _ in range(5):
        oracle.run(p, f_or, 1)
        f_bf = step(f_bf, prm)
        scale = np.abs(f_bf).max()
        assert np.abs(f_or - f_bf).max() <= 1e-13 * scale


def test_body_force_term_matches_brute_force(oracle_lib):
    oracle, p, prm, f0 = _case(9, 8, False, seed=5, F0=1e-4)
    f_or = f0.copy()
    oracle.run(p, f_or, 3)
    f_bf = f0.copy()
    for _ in range(3):
        f_bf = step(f_bf, prm)
    assert np.abs(f_or - f_bf).max() <= 1e-13 * np.abs(f_bf).max()
    # and the term matters: without it the results differ far above rounding
    prm0 = dict(prm, F0=0.0)
    f_nf = f0.copy()
    for _ in range(3):
        f_nf = step(f_nf, prm0)
    assert np.abs(f_or - f_nf).max() > 1e-8


def test_a_planted_mistake_is_caught(oracle_lib):
    """The comparison has teeth: flipping the sign of one repulsion shell in
    the brute force changes the result far above the tolerance."""
    oracle, p, prm, f0 = _case(8, 8, False, seed=3)
    f_or = f0.copy()
    oracle.run(p, f_or, 2)
    bad = dict(prm, Gr=(-11.70, 10.95))
    f_bad = f0.copy()
    for _ in range(2):
        f_bad = step(f_bad, bad)
    assert np.abs(f_or - f_bad).max() > 1e-6


def readouts(f, prm, half_force=True):
    """Every read-out of the state f at time t, from the definitions:
    physical velocity u = (sum_s j_s + F_s/2) / sum_s rho_s; deviatoric
    stress sigma_xy = -sum_s (1 - 1/(2 tau_s)) sum_i c_ix c_iy (f_is -
    f^eq_i(rho_s, u)); lattice totals; row means; the Kolmogorov-mode
    amplitude of u_x and grad rho_A . grad rho_B with the D2Q9 gradient
    3 sum_i w_i c_i rho(x + c_i) (neighbours wrapped, or mirrored at walls)."""
    W, _, _ = _weights()
    ny, nx = f.shape[2:]
    rho, jx, jy, F = forces(f, prm)
    h = 0.5 if half_force else 0.0
    rt = rho.sum(axis=0)
    ux = (jx.sum(axis=0) + h * F[:, 0].sum(axis=0)) / rt
    uy = (jy.sum(axis=0) + h * F[:, 1].sum(axis=0)) / rt
    sxy = np.zeros((ny, nx))
    for s in range(2):
        neq = f[s] - feq_all(W, rho[s], ux, uy)
        sxy -= (1.0 - 0.5 / prm["tau"][s]) * np.tensordot(CX * CY, neq, axes=([0], [0]))
    y = np.arange(ny)[:, None]
    u_bar = 2.0 / (nx * ny) * float((ux * np.sin(2.0 * np.pi * y / ny)).sum())
    grads = []
    for s in range(2):
        gx = sum(3.0 * W[i] * CX[i] * _shift(rho[s], CX[i], CY[i], prm["walls"]) for i in range(9))
        gy = sum(3.0 * W[i] * CY[i] * _shift(rho[s], CX[i], CY[i], prm["walls"]) for i in range(9))
        grads.append((gx, gy))
    i_ab = float((grads[0][0] * grads[1][0] + grads[0][1] * grads[1][1]).sum())
    mom = (jx.sum(axis=0) + 0.5 * F[:, 0].sum(axis=0)).sum(), \
        (jy.sum(axis=0) + 0.5 * F[:, 1].sum(axis=0)).sum()
    return dict(rho=rho, ux=ux, uy=uy, sxy=sxy, mass=rho.sum(axis=(1, 2)), mom=np.array(mom),
                sxy_total=sxy.sum(), ux_row=ux.mean(axis=1), sxy_row=sxy.mean(axis=1),
                u_bar=u_bar, i_ab=i_ab)


@pytest.mark.parametrize("forcing", ["shift", "guo"])
@pytest.mark.parametrize("walls", [False, True])
def test_readouts_match_brute_force(oracle_lib, walls, forcing):
    """Moments (with the half-force velocity), sigma_xy, totals, row
    profiles, u_bar and I_AB of an evolved state with forces and a body
    force on, against the definitions evaluated on whole arrays."""
    nx, ny = 9, 8
    oracle, p, prm, f = _case(nx, ny, walls, seed=17, F0=3e-3,
                              wall_u=(0.01, -0.04) if walls else (0.0, 0.0), forcing=forcing)
    oracle.run(p, f, 4)
    bf = readouts(f, prm)
    r, ux, uy = oracle.moments(p, f)
    tol = 1e-13
    assert np.abs(r - bf["rho"]).max() <= tol
    assert np.abs(ux - bf["ux"]).max() <= tol and np.abs(uy - bf["uy"]).max() <= tol
    tot = oracle.totals(p, f)
    assert np.allclose(tot["mass"], bf["mass"], rtol=1e-14, atol=0)
    assert np.abs(tot["mom"] - bf["mom"]).max() <= 1e-12
    assert abs(tot["sxy"] - bf["sxy_total"]) <= 1e-12
    ux_row, sxy_row = oracle.row_profiles(p, f)
    assert np.abs(ux_row - bf["ux_row"]).max() <= tol
    assert np.abs(sxy_row - bf["sxy_row"]).max() <= tol
    assert np.abs(sxy_row).max() > 1e-4          # the stress read-out is exercised
    sf = oracle.shear_flow(p, f)
    assert abs(sf["u_bar"] - bf["u_bar"]) <= tol
    assert abs(sf["i_ab"] - bf["i_ab"]) <= 1e-12 * max(1.0, abs(bf["i_ab"]))
    # the half-force term is visible at this size: dropping it is caught
    no_half = readouts(f, prm, half_force=False)
    assert np.abs(ux - no_half["ux"]).max() > 1e-6


@pytest.mark.parametrize("walls", [False, True])
def test_init_is_the_equilibrium_of_the_given_fields(oracle_lib, walls):
    """f_is(x, 0) = f^eq_i(rho_s(x), u(x)) at every site, in the oracle's
    [s][i][y][x] layout (the step tests start both sides from this state, so
    they cannot see a mistake in it)."""
    import oracle
    W, _, _ = _weights()
    nx, ny = 7, 6
    p = oracle.Params(nx=nx, ny=ny, walls=walls)
    rho = inputs.random_densities(nx, ny, 23, amp=0.3)
    rng = np.random.default_rng(23)
    ux, uy = 0.1 * rng.standard_normal((2, ny, nx))
    f = oracle.init(p, rho, ux, uy)
    assert f.shape == (2, 9, ny, nx)
    for s in range(2):
        assert np.abs(f[s] - feq_all(W, rho[s], ux, uy)).max() <= 1e-15
    f0 = oracle.init(p, rho)                     # velocity omitted: at rest
    for s in range(2):
        assert np.abs(f0[s] - feq_all(W, rho[s], 0.0 * ux, 0.0 * uy)).max() <= 1e-15
