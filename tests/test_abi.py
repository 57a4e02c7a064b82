"""The C ABI without a GPU: the library loads, exports every function that
include/sclbm.h declares, and rejects invalid input before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sclbm.h")


@pytest.fixture(scope="module")
def L():
    from paper_0807_4471_amd import sclbm
    return sclbm


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sclbm_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(L):
    names = declared()
    assert len(names) >= 20
    raw = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in names if not hasattr(raw, n)]
    assert not missing, missing


def test_index_selftest(L):
    """Row folding used by the kernels: every staged row lands in the lattice."""
    assert L.lib.sclbm_selftest() == 0


def test_diag_record_matches_header(L):
    """The binding's diagnostics record has the header's size and field order."""
    import ctypes as C
    names = [n for n, _ in L.Diag._fields_]
    assert names == ["mass", "mom", "sxy", "wall_mom", "wall_steps", "step", "bad_sites",
                     "u_bar", "i_ab"]
    assert C.sizeof(L.Diag) == 8 * (2 + 2 + 1 + 4 + 3 + 2)


def test_version_and_strerror(L):
    assert L.lib.sclbm_abi_version() == 2
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.strerror(code) and L.strerror(code) != "unknown status"
    assert L.strerror(-99) == "unknown status"


def test_state_bytes_scaling(L):
    a = L.state_bytes(L.make_desc(512, 512, storage="f32"))
    b = L.state_bytes(L.make_desc(512, 512, storage="f16dev"))
    c = L.state_bytes(L.make_desc(512, 512, storage="f64"))
    pop32 = 2 * 18 * 512 * 512 * 4
    assert pop32 <= a < pop32 * 1.05
    assert b < a < c
    w = L.state_bytes(L.make_desc(512, 512, storage="f32", boundary="walls"))
    assert w > a          # two ghost rows


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(ny=-1), dict(nx=70000), dict(tau=(0.5, 1.0)), dict(tau=(1.0, float("nan"))),
    dict(rho0=0.0), dict(psi_amp=-1.0), dict(Gx=float("inf")), dict(diag_every=-2),
    dict(boundary=7), dict(storage=9), dict(boundary="walls", ny=1),
    dict(storage="f16dev", rho_ref=(float("nan"), 0.7)), dict(forcing=2), dict(forcing=-1),
])
def test_invalid_descriptors(L, bad):
    kw = dict(nx=32, ny=32)
    kw.update(bad)
    d = L.make_desc(**kw)
    assert L.state_bytes(d) == 0
    h = ctypes.c_void_p()
    rc = L.lib.sclbm_bind(ctypes.byref(d), ctypes.c_void_p(1 << 20), 1 << 30, ctypes.byref(h))
    assert rc == L.EINVAL and not h.value
    assert L.last_error()


def test_bind_errors_and_state(L):
    d = L.make_desc(100, 60, storage="f32")
    need = L.state_bytes(d)
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)          # never dereferenced by bind
    assert L.lib.sclbm_bind(ctypes.byref(d), fake, need - 1, ctypes.byref(h)) == L.ESIZE
    assert L.lib.sclbm_bind(ctypes.byref(d), None, need, ctypes.byref(h)) == L.EINVAL
    assert L.lib.sclbm_bind(ctypes.byref(d), ctypes.c_void_p((1 << 20) + 8), need,
                            ctypes.byref(h)) == L.EINVAL
    assert L.lib.sclbm_bind(ctypes.byref(d), fake, need, None) == L.EINVAL
    assert L.lib.sclbm_bind(ctypes.byref(d), fake, need, ctypes.byref(h)) == L.OK
    try:
        # not initialised: no device work may be enqueued
        assert L.lib.sclbm_step(h, 1, None) == L.ESTATE
        assert L.lib.sclbm_read_moments(h, None, None, None, None, None, None) == L.ESTATE
        assert L.lib.sclbm_step(h, -1, None) in (L.ESTATE, L.EINVAL)
        t = L.Tiling()
        assert L.lib.sclbm_get_tiling(h, ctypes.byref(t)) == L.OK
        assert (t.stacked == 0 and t.waves in (1, 2, 4) and t.tile_x <= 64 * t.waves - 4) or \
            (t.stacked == 1 and t.waves in (4, 8) and t.tile_x <= 60)
        for bad in [(61, 8, 1, 0), (60, 8, 3, 0), (20, 8, 1, 0), (60, 3, 1, 0), (253, 8, 4, 0),
                    (60, 8, 4, 1), (61, 8, 8, 1), (60, 8, 2, 1), (60, 8, 8, 2),
                    (60, 8, 1, 0, 2), (60, 8, 1, 0, 0, 1)]:
            tb = L.Tiling(*bad)
            assert L.lib.sclbm_set_tiling(h, ctypes.byref(tb)) == L.EINVAL, bad
        ok = L.Tiling(100, 8, 2, 0)
        assert L.lib.sclbm_set_tiling(h, ctypes.byref(ok)) == L.OK
        assert L.lib.sclbm_get_tiling(h, ctypes.byref(t)) == L.OK
        assert (t.tile_x, t.tile_y, t.waves, t.stacked, t.throttle) == (100, 8, 2, 0, 0)
        ok = L.Tiling(50, 8, 8, 1)
        assert L.lib.sclbm_set_tiling(h, ctypes.byref(ok)) == L.OK
        wt = L.Tiling(50, 4, 4, 1, 0, 1)
        assert L.lib.sclbm_set_tiling(h, ctypes.byref(wt)) == L.OK
        assert L.lib.sclbm_get_tiling(h, ctypes.byref(t)) == L.OK and t.write_through == 1
        for bad in [(50, 4, 4, 1, 0, 2), (100, 8, 2, 0, 0, 1)]:
            assert L.lib.sclbm_set_tiling(h, ctypes.byref(L.Tiling(*bad))) == L.EINVAL, bad
        v = ctypes.c_int64(-5)
        assert L.lib.sclbm_time(h, ctypes.byref(v)) == L.OK
        assert L.lib.sclbm_checkpoint_bytes(h) > 0
        assert L.lib.sclbm_restore(h, ctypes.create_string_buffer(8), 8, None) == L.ESIZE
    finally:
        assert L.lib.sclbm_release(h) == L.OK
    assert L.lib.sclbm_release(None) == L.OK


def test_forcing_names(L):
    assert L.make_desc(8, 8, forcing="guo").forcing == 1
    assert L.make_desc(8, 8).forcing == 0
    assert L.state_bytes(L.make_desc(8, 8, forcing="guo")) == L.state_bytes(L.make_desc(8, 8))
    with pytest.raises(ValueError):
        L.make_desc(8, 8, forcing="he")


@pytest.mark.parametrize("storage,eb,largest", [("f64", 8, 5440), ("f32", 4, 7703),
                                                ("f16dev", 2, 10901)])
def test_largest_square_lattice(L, storage, eb, largest):
    """32-bit offsets: the 9 planes of a species (rows padded to 64
    elements, plus 128 elements per plane) must span < 2 GiB; the largest
    accepted square lattice is the last one that fits, the next is
    EUNSUPPORTED."""
    def fits(n):
        return 9 * ((n + 63) // 64 * 64 * n + 128) * eb < 2 ** 31
    assert fits(largest) and not fits(largest + 1)
    assert L.state_bytes(L.make_desc(largest, largest, storage=storage)) > 0
    d = L.make_desc(largest + 1, largest + 1, storage=storage)
    assert L.state_bytes(d) == 0
    h = ctypes.c_void_p()
    rc = L.lib.sclbm_bind(ctypes.byref(d), ctypes.c_void_p(1 << 20), 1 << 40, ctypes.byref(h))
    assert rc == L.EUNSUPPORTED and not h.value


def test_batch_rejects_a_repeated_instance(L):
    """One state named twice in a batch would be stepped twice per launch
    (racing) and have its time and ping-pong copy advanced twice: refused
    before any device work."""
    d = L.make_desc(64, 64, storage="f32")
    need = L.state_bytes(d)
    hs = [ctypes.c_void_p(), ctypes.c_void_p()]
    for k, h in enumerate(hs):
        fake = ctypes.c_void_p((1 << 30) * (k + 1))   # never dereferenced
        assert L.lib.sclbm_bind(ctypes.byref(d), fake, need, ctypes.byref(h)) == L.OK
    try:
        tl = (L.Tiling * 2)(L.Tiling(60, 4, 4, 1), L.Tiling(60, 4, 4, 1))
        two = (ctypes.c_void_p * 2)(hs[0].value, hs[1].value)
        same = (ctypes.c_void_p * 2)(hs[0].value, hs[0].value)
        assert L.lib.sclbm_batch_bytes(two, 2, tl) > 0
        assert L.lib.sclbm_batch_bytes(same, 2, tl) == 0
        assert "twice" in L.last_error()
        out = ctypes.c_void_p()
        ws = ctypes.c_void_p(1 << 34)
        assert L.lib.sclbm_batch_plan(same, 2, tl, ws, 1 << 20, None,
                                      ctypes.byref(out)) == L.EINVAL
        assert out.value is None
    finally:
        for h in hs:
            L.lib.sclbm_release(h)


def test_static_batch_rejects_before_device_work(L):
    """sclbm_batch_step_static refuses, before any device work: tables larger
    than its static array (ESIZE), a repeated instance, NULL steps."""
    d = L.make_desc(8192, 4096, storage="f16dev")
    need = L.state_bytes(d)
    hs = [ctypes.c_void_p() for _ in range(3)]
    for k, h in enumerate(hs):
        fake = ctypes.c_void_p((1 << 34) * (k + 1))   # never dereferenced
        assert L.lib.sclbm_bind(ctypes.byref(d), fake, need, ctypes.byref(h)) == L.OK
    try:
        # stacked 32 x 4 tiles: 256 x 1024 tiles per instance, 6 MiB of tables
        tl = (L.Tiling * 3)(*[L.Tiling(32, 4, 4, 1) for _ in range(3)])
        arr = (ctypes.c_void_p * 3)(*[h.value for h in hs])
        steps = (ctypes.c_int64 * 3)(1, 1, 1)
        assert L.lib.sclbm_batch_step_static(arr, 3, tl, steps, None) == L.ESIZE
        assert "static scratch" in L.last_error()
        same = (ctypes.c_void_p * 2)(hs[0].value, hs[0].value)
        assert L.lib.sclbm_batch_step_static(same, 2, tl, steps, None) == L.EINVAL
        assert L.lib.sclbm_batch_step_static(arr, 3, tl, None, None) == L.EINVAL
        # fits, but the instances were never initialised: refused as well
        one = (ctypes.c_void_p * 1)(hs[0].value)
        assert L.lib.sclbm_batch_step_static(one, 1, tl, steps, None) == L.ESTATE
    finally:
        for h in hs:
            L.lib.sclbm_release(h)
