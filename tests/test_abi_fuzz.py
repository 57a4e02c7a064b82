"""Descriptor validation under random input (no GPU): for any descriptor the
library either refuses it (state_bytes 0, bind EINVAL or EUNSUPPORTED, no
handle) or accepts it (state_bytes > 0, bind OK with a buffer of exactly
that size, ESIZE with one byte less), and what it accepts is what the
header's rules allow: sizes in range, tau > 1/2, finite couplings,
rho0 > 0, psi_amp > 0, the 2 GiB plane rule."""
import ctypes
import math

import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st


@pytest.fixture(scope="module")
def L():
    from paper_0807_4471_amd import sclbm
    return sclbm


finite = st.floats(min_value=-20.0, max_value=20.0, allow_nan=False)
anyf = st.one_of(finite, st.sampled_from([float("nan"), float("inf"), -float("inf"), 0.0, 0.5]))


def expected_ok(nx, ny, boundary, storage, tau, Ga, Gr, Gx, rho0, psi, rho_ref, wall_u, F0, K):
    if not (1 <= nx <= 65536 and 1 <= ny <= 65536) or nx * ny > 2 ** 31 - 1:
        return False
    if boundary == 1 and ny < 2:
        return False
    ok = all(math.isfinite(t) and t > 0.5 for t in tau)
    ok &= all(math.isfinite(g) for g in (*Ga, *Gr, Gx, F0))
    ok &= math.isfinite(rho0) and rho0 > 0 and math.isfinite(psi) and psi > 0 and K >= 0
    if storage in (2, 3):
        ok &= all(math.isfinite(r) and r >= 0 for r in rho_ref)
    if boundary == 1:
        ok &= all(math.isfinite(u) for u in wall_u)
    if not ok:
        return False
    eb = {0: 8, 1: 4, 2: 2, 3: 2}[storage]
    rows = ny + (2 if boundary == 1 else 0)
    return 9 * (((nx + 63) // 64 * 64) * rows + 128) * eb < 2 ** 31


@settings(max_examples=400, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(nx=st.integers(-3, 12000), ny=st.integers(-3, 12000), boundary=st.sampled_from([0, 1]),
       storage=st.sampled_from([0, 1, 2, 3]), tau=st.tuples(anyf, anyf),
       Ga=st.tuples(anyf, anyf), Gr=st.tuples(finite, finite), Gx=anyf,
       rho0=anyf, psi=anyf, rho_ref=st.tuples(anyf, anyf), wall_u=st.tuples(anyf, anyf),
       F0=anyf, K=st.integers(-2, 100))
def test_random_descriptors(L, nx, ny, boundary, storage, tau, Ga, Gr, Gx, rho0, psi, rho_ref,
                            wall_u, F0, K):
    d = L.make_desc(nx, ny, storage=storage, boundary=boundary, tau=tau, Ga=Ga, Gr=Gr, Gx=Gx,
                    rho0=rho0, psi_amp=psi, rho_ref=rho_ref, wall_u=wall_u, body_F0=F0,
                    diag_every=K)
    want = expected_ok(nx, ny, boundary, storage, tau, Ga, Gr, Gx, rho0, psi, rho_ref, wall_u,
                       F0, K)
    need = L.state_bytes(d)
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)            # never dereferenced by bind
    if not want:
        assert need == 0
        rc = L.lib.sclbm_bind(ctypes.byref(d), fake, 1 << 40, ctypes.byref(h))
        assert rc in (L.EINVAL, L.EUNSUPPORTED) and not h.value
        return
    assert need > 0
    assert L.lib.sclbm_bind(ctypes.byref(d), fake, need - 1, ctypes.byref(h)) == L.ESIZE
    assert not h.value
    assert L.lib.sclbm_bind(ctypes.byref(d), fake, need, ctypes.byref(h)) == L.OK and h.value
    assert L.lib.sclbm_release(h) == L.OK


def expected_tiling_ok(nx, ny, W, H, waves, stacked, throttle, wt):
    if stacked not in (0, 1) or throttle not in (0, 1) or wt not in (0, 1):
        return False
    if wt and not stacked:
        return False
    if stacked:
        if waves not in (4, 8) or H != waves or W > 60:
            return False
    else:
        if waves not in (1, 2, 4) or W > 64 * waves - 4 or H < min(4, ny):
            return False
    return W >= min(32, nx)


@settings(max_examples=400, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(nx=st.integers(1, 600), ny=st.integers(2, 600), W=st.integers(-5, 300),
       H=st.integers(-5, 300), waves=st.integers(-1, 9), stacked=st.integers(-1, 2),
       throttle=st.integers(-1, 2), wt=st.integers(-1, 2))
def test_random_tilings(L, nx, ny, W, H, waves, stacked, throttle, wt):
    """sclbm_set_tiling accepts exactly the tilings the header's rules allow,
    and a refused one leaves the current tiling in place."""
    d = L.make_desc(nx, ny, storage="f32")
    need = L.state_bytes(d)
    h = ctypes.c_void_p()
    assert L.lib.sclbm_bind(ctypes.byref(d), ctypes.c_void_p(1 << 20), need,
                            ctypes.byref(h)) == L.OK
    try:
        before = L.Tiling()
        assert L.lib.sclbm_get_tiling(h, ctypes.byref(before)) == L.OK
        rc = L.lib.sclbm_set_tiling(h, ctypes.byref(L.Tiling(W, H, waves, stacked, throttle, wt)))
        after = L.Tiling()
        assert L.lib.sclbm_get_tiling(h, ctypes.byref(after)) == L.OK
        got = (after.tile_x, after.tile_y, after.waves, after.stacked, after.throttle,
               after.write_through)
        if expected_tiling_ok(nx, ny, W, H, waves, stacked, throttle, wt):
            assert rc == L.OK and got == (W, H, waves, stacked, throttle, wt)
        else:
            assert rc == L.EINVAL
            assert got == (before.tile_x, before.tile_y, before.waves, before.stacked,
                           before.throttle, before.write_through)
    finally:
        L.lib.sclbm_release(h)
