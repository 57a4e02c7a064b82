"""ctypes binding of the plain FP64 CPU oracle (``oracle/sclbm_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``bench.py`` (its
``cpu_baseline`` leg) and ``__graft_entry__.smoke()``.  The product package
never imports this module, and this module imports nothing from the product
package.

Array conventions (numpy float64, C order):
  f    (2, 9, ny, nx)   post-streaming populations f_is(r, t) of Eq. (1)
  rho  (2, ny, nx)      species densities
  psi  (2, ny, nx)      pseudo-potential fields
  F    (2, 2, ny, nx)   force per species and component (x, y)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sclbm_oracle.c")
_LIB = os.path.join(_HERE, "libsclbm_oracle.so")

# -fopenmp: rows of a step run in parallel (same arithmetic for any thread count)
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c99",
          "-fopenmp"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc; returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("walls", ctypes.c_int32), ("forcing", ctypes.c_int32),
        ("tau", ctypes.c_double * 2),
        ("Ga", ctypes.c_double * 2),
        ("Gr", ctypes.c_double * 2),
        ("Gx", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("psi_amp", ctypes.c_double),
        ("wall_u", ctypes.c_double * 2),
        ("body_F0", ctypes.c_double),
    ]


@dataclass
class Params:
    """Physical parameters of one lattice (defaults: the 64x64 FP64 case)."""
    nx: int = 64
    ny: int = 64
    walls: bool = False
    tau: tuple = (1.0, 1.0)
    Ga: tuple = (-12.55, -11.80)
    Gr: tuple = (11.70, 10.95)
    Gx: float = 0.58
    rho0: float = 0.70
    psi_amp: float | None = None      # None -> rho0 (amplitude used by the workloads)
    wall_u: tuple = (0.0, 0.0)
    body_F0: float = 0.0
    forcing: str = "shift"            # "shift" (Shan-Chen velocity shift) or "guo"

    def c(self) -> _Params:
        amp = self.rho0 if self.psi_amp is None else self.psi_amp
        return _Params(int(self.nx), int(self.ny), int(bool(self.walls)),
                       {"shift": 0, "guo": 1}[self.forcing],
                       (ctypes.c_double * 2)(*self.tau),
                       (ctypes.c_double * 2)(*self.Ga),
                       (ctypes.c_double * 2)(*self.Gr),
                       float(self.Gx), float(self.rho0), float(amp),
                       (ctypes.c_double * 2)(*self.wall_u), float(self.body_F0))


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        pp = ctypes.POINTER(_Params)
        L.oracle_d2q9.argtypes = [ip, ip, dp]
        L.oracle_d2q9.restype = None
        L.oracle_stencil.argtypes = [ip, ip, dp, dp, dp, dp]
        L.oracle_stencil.restype = None
        L.oracle_psi.argtypes = [pp, ctypes.c_double]
        L.oracle_psi.restype = ctypes.c_double
        L.oracle_feq.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.oracle_feq.restype = None
        L.oracle_forces.argtypes = [pp, dp, dp, dp]
        L.oracle_init.argtypes = [pp, dp, dp, dp, dp]
        L.oracle_run.argtypes = [pp, dp, ctypes.c_int64, dp]
        L.oracle_moments.argtypes = [pp, dp, dp, dp, dp]
        L.oracle_totals.argtypes = [pp, dp, dp]
        L.oracle_row_profiles.argtypes = [pp, dp, dp, dp]
        L.oracle_shear_flow.argtypes = [pp, dp, dp]
        L.oracle_set_threads.argtypes = [ctypes.c_int32]
        L.oracle_set_threads.restype = ctypes.c_int32
        L.oracle_threads.argtypes = []
        L.oracle_threads.restype = ctypes.c_int32
        for name in ("oracle_forces", "oracle_init", "oracle_run", "oracle_moments",
                     "oracle_totals", "oracle_row_profiles", "oracle_shear_flow"):
            getattr(L, name).restype = ctypes.c_int32
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def set_threads(n: int) -> int:
    """Threads of the oracle's row loops (n < 1: all processors); returns the
    number set.  Results do not depend on it."""
    return int(lib().oracle_set_threads(int(n)))


def threads() -> int:
    return int(lib().oracle_threads())


def d2q9():
    cx = (ctypes.c_int32 * 9)()
    cy = (ctypes.c_int32 * 9)()
    w = (ctypes.c_double * 9)()
    lib().oracle_d2q9(cx, cy, w)
    return np.array(cx[:]), np.array(cy[:]), np.array(w[:])


def stencil():
    """(ex, ey, wa, wr, w0, p0) of the 24 force offsets."""
    ex = (ctypes.c_int32 * 24)()
    ey = (ctypes.c_int32 * 24)()
    wa = (ctypes.c_double * 24)()
    wr = (ctypes.c_double * 24)()
    w0 = ctypes.c_double()
    p0 = ctypes.c_double()
    lib().oracle_stencil(ex, ey, wa, wr, ctypes.byref(w0), ctypes.byref(p0))
    return (np.array(ex[:]), np.array(ey[:]), np.array(wa[:]), np.array(wr[:]),
            w0.value, p0.value)


def psi(p: Params, rho: float) -> float:
    return lib().oracle_psi(ctypes.byref(p.c()), float(rho))


def feq(rho: float, ux: float, uy: float) -> np.ndarray:
    out = np.zeros(9)
    lib().oracle_feq(float(rho), float(ux), float(uy), _ptr(out))
    return out


def forces(p: Params, psi_f: np.ndarray, rho_f: np.ndarray) -> np.ndarray:
    psi_f = np.ascontiguousarray(psi_f, dtype=np.float64)
    rho_f = np.ascontiguousarray(rho_f, dtype=np.float64)
    assert psi_f.shape == (2, p.ny, p.nx) and rho_f.shape == (2, p.ny, p.nx)
    F = np.zeros((2, 2, p.ny, p.nx))
    _check(lib().oracle_forces(ctypes.byref(p.c()), _ptr(psi_f), _ptr(rho_f), _ptr(F)), "forces")
    return F


def init(p: Params, rho: np.ndarray, ux=None, uy=None) -> np.ndarray:
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    assert rho.shape == (2, p.ny, p.nx)
    ux = None if ux is None else np.ascontiguousarray(ux, dtype=np.float64)
    uy = None if uy is None else np.ascontiguousarray(uy, dtype=np.float64)
    f = np.zeros((2, 9, p.ny, p.nx))
    _check(lib().oracle_init(ctypes.byref(p.c()), _ptr(rho), _ptr(ux), _ptr(uy), _ptr(f)), "init")
    return f


def run(p: Params, f: np.ndarray, nsteps: int, wall_mom: np.ndarray | None = None) -> np.ndarray:
    """Advance f (in place) by nsteps; wall momentum is added into wall_mom (2, 2)."""
    assert f.shape == (2, 9, p.ny, p.nx) and f.dtype == np.float64 and f.flags["C_CONTIGUOUS"]
    if wall_mom is not None:
        assert wall_mom.shape == (2, 2) and wall_mom.dtype == np.float64
    _check(lib().oracle_run(ctypes.byref(p.c()), _ptr(f), int(nsteps), _ptr(wall_mom)), "run")
    return f


def moments(p: Params, f: np.ndarray):
    """(rho (2,ny,nx), ux (ny,nx), uy (ny,nx)) at the time of f."""
    rho = np.zeros((2, p.ny, p.nx))
    ux = np.zeros((p.ny, p.nx))
    uy = np.zeros((p.ny, p.nx))
    _check(lib().oracle_moments(ctypes.byref(p.c()), _ptr(f), _ptr(rho), _ptr(ux), _ptr(uy)),
           "moments")
    return rho, ux, uy


def totals(p: Params, f: np.ndarray) -> dict:
    out = np.zeros(6)
    _check(lib().oracle_totals(ctypes.byref(p.c()), _ptr(f), _ptr(out)), "totals")
    return {"mass": out[0:2].copy(), "mom": out[2:4].copy(), "sxy": out[4],
            "bad": int(out[5])}


def row_profiles(p: Params, f: np.ndarray):
    ux = np.zeros(p.ny)
    sxy = np.zeros(p.ny)
    _check(lib().oracle_row_profiles(ctypes.byref(p.c()), _ptr(f), _ptr(ux), _ptr(sxy)),
           "row_profiles")
    return ux, sxy


def shear_flow(p: Params, f: np.ndarray) -> dict:
    """U_bar (sin-mode amplitude of the physical x-velocity) and I_AB."""
    out = np.zeros(2)
    _check(lib().oracle_shear_flow(ctypes.byref(p.c()), _ptr(f), _ptr(out)), "shear_flow")
    return {"u_bar": float(out[0]), "i_ab": float(out[1])}
