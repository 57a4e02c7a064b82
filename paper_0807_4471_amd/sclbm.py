"""ctypes binding of libsclbm.so (include/sclbm.h).

Argument marshalling only: every step of the lattice Boltzmann path runs in
the HIP kernels of the library.  PyTorch provides device memory (the state
buffer is a ``torch.uint8`` CUDA tensor) and the HIP stream
(``torch.cuda.current_stream()``).  Importing this module loads the library
and raises if it is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SCLBM_LIBRARY selects another build of the same library (the tests use it
# for the NaN-poisoned-LDS debug build); default: the in-tree libsclbm.so.
LIB_PATH = os.environ.get("SCLBM_LIBRARY") or os.path.join(_HERE, "libsclbm.so")

OK, EINVAL, ESIZE, EDEVICE, ENONFINITE, EUNSUPPORTED, ESTATE = 0, -1, -2, -3, -4, -5, -6
PERIODIC, WALLS_Y = 0, 1
F64, F32, F16DEV, F16DEV_SR = 0, 1, 2, 3
STORAGE = {"f64": F64, "f32": F32, "f16dev": F16DEV, "f16sr": F16DEV_SR}
BOUNDARY = {"periodic": PERIODIC, "walls": WALLS_Y}
BYTES_PER_POP = {F64: 8, F32: 4, F16DEV: 2, F16DEV_SR: 2}
FORCING = {"shift": 0, "guo": 1}


class Desc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("boundary", ctypes.c_int32), ("storage", ctypes.c_int32),
        ("tau", ctypes.c_double * 2),
        ("G_a", ctypes.c_double * 2),
        ("G_r", ctypes.c_double * 2),
        ("G_x", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("psi_amp", ctypes.c_double),
        ("rho_ref", ctypes.c_double * 2),
        ("wall_u", ctypes.c_double * 2),
        ("body_F0", ctypes.c_double),
        ("diag_every", ctypes.c_int32),
        ("forcing", ctypes.c_int32),
    ]


class Diag(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double * 2),
        ("mom", ctypes.c_double * 2),
        ("sxy", ctypes.c_double),
        ("wall_mom", (ctypes.c_double * 2) * 2),
        ("wall_steps", ctypes.c_int64),
        ("step", ctypes.c_int64),
        ("bad_sites", ctypes.c_int64),
        ("u_bar", ctypes.c_double),
        ("i_ab", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {"mass": np.array(self.mass[:]), "mom": np.array(self.mom[:]), "sxy": self.sxy,
                "wall_mom": np.array([[self.wall_mom[w][c] for c in range(2)] for w in range(2)]),
                "wall_steps": int(self.wall_steps), "step": int(self.step),
                "bad_sites": int(self.bad_sites), "u_bar": float(self.u_bar),
                "i_ab": float(self.i_ab)}


class Tiling(ctypes.Structure):
    _fields_ = [("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32),
                ("waves", ctypes.c_int32), ("stacked", ctypes.c_int32),
                ("throttle", ctypes.c_int32), ("write_through", ctypes.c_int32)]


class SclbmError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} ({status}): {last_error()}")


def _load():
    # torch ships its own HIP runtime (SONAME libamdhip64.so.7).  Loading torch
    # first makes libsclbm.so bind to that same runtime, so device buffers and
    # streams from torch are valid in the library.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_0807_4471_amd.build` (no fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    vp, dp, i32, i64, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int32, \
        ctypes.c_int64, ctypes.c_size_t
    pd = ctypes.POINTER(Desc)
    sig = {
        "sclbm_abi_version": ([], i32),
        "sclbm_selftest": ([], i32),
        "sclbm_strerror": ([i32], ctypes.c_char_p),
        "sclbm_last_error": ([], ctypes.c_char_p),
        "sclbm_state_bytes": ([pd], sz),
        "sclbm_bind": ([pd, vp, sz, ctypes.POINTER(vp)], i32),
        "sclbm_init_random": ([vp, ctypes.c_uint64, dp, ctypes.c_double, vp], i32),
        "sclbm_init_fields": ([vp, vp, vp, vp, vp, vp], i32),
        "sclbm_step": ([vp, i64, vp], i32),
        "sclbm_time": ([vp, ctypes.POINTER(i64)], i32),
        "sclbm_set_tiling": ([vp, ctypes.POINTER(Tiling)], i32),
        "sclbm_get_tiling": ([vp, ctypes.POINTER(Tiling)], i32),
        "sclbm_read_moments": ([vp, vp, vp, vp, vp, vp, vp], i32),
        "sclbm_order_parameter": ([vp, vp, vp, dp, vp], i32),
        "sclbm_diagnostics": ([vp, ctypes.POINTER(Diag), vp], i32),
        "sclbm_fused_diagnostics": ([vp, ctypes.POINTER(Diag), vp], i32),
        "sclbm_reset_wall_accum": ([vp, vp], i32),
        "sclbm_checkpoint_bytes": ([vp], sz),
        "sclbm_checkpoint": ([vp, vp, sz, vp], i32),
        "sclbm_restore": ([vp, vp, sz, vp], i32),
        "sclbm_release": ([vp], i32),
        "sclbm_batch_bytes": ([ctypes.POINTER(vp), i32, ctypes.POINTER(Tiling)], sz),
        "sclbm_batch_plan": ([ctypes.POINTER(vp), i32, ctypes.POINTER(Tiling), vp, sz, vp,
                              ctypes.POINTER(vp)], i32),
        "sclbm_batch_step": ([vp, ctypes.POINTER(i64), vp], i32),
        "sclbm_batch_status": ([vp, vp], i32),
        "sclbm_batch_release": ([vp], i32),
        "sclbm_batch_info": ([vp, ctypes.POINTER(i32)], i32),
        "sclbm_batch_set_mode": ([vp, i32], i32),
        "sclbm_batch_set_barrier_limit": ([vp, ctypes.c_uint32], i32),
        "sclbm_batch_step_static": ([ctypes.POINTER(vp), i32, ctypes.POINTER(Tiling),
                                     ctypes.POINTER(i64), vp], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


lib = _load()


def strerror(status: int) -> str:
    return lib.sclbm_strerror(status).decode()


def last_error() -> str:
    return lib.sclbm_last_error().decode()


def check(status: int, what: str) -> int:
    if status != OK:
        raise SclbmError(status, what)
    return status


def make_desc(nx, ny, storage="f32", boundary="periodic", tau=(1.0, 1.0),
              Ga=(-12.55, -11.80), Gr=(11.70, 10.95), Gx=0.58, rho0=0.70, psi_amp=None,
              rho_ref=(0.7, 0.7), wall_u=(0.0, 0.0), body_F0=0.0, diag_every=0,
              forcing="shift") -> Desc:
    """Descriptor; defaults are the workload couplings with Psi amplitude rho0.
    forcing: "shift" (Shan-Chen equilibrium-velocity shift) or "guo"."""
    if isinstance(forcing, str) and forcing not in FORCING:
        raise ValueError(f"forcing must be one of {list(FORCING)}")
    return Desc(int(nx), int(ny), BOUNDARY.get(boundary, boundary), STORAGE.get(storage, storage),
                (ctypes.c_double * 2)(*tau), (ctypes.c_double * 2)(*Ga),
                (ctypes.c_double * 2)(*Gr), float(Gx), float(rho0),
                float(rho0 if psi_amp is None else psi_amp),
                (ctypes.c_double * 2)(*rho_ref), (ctypes.c_double * 2)(*wall_u),
                float(body_F0), int(diag_every), FORCING.get(forcing, forcing))


def state_bytes(desc: Desc) -> int:
    return int(lib.sclbm_state_bytes(ctypes.byref(desc)))


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Simulation:
    """One lattice whose state lives in a caller-owned (torch) device buffer."""

    def __init__(self, nx: int, ny: int, device="cuda", buffer=None, tiling=None, **kw):
        """tiling: None (library default), "auto" (the autotuner's table for
        this architecture, if it has an entry or a nearby size), or a tuple
        (tile_x, tile_y, waves[, stacked[, throttle]])."""
        import torch
        self.desc = make_desc(nx, ny, **kw)
        self.nx, self.ny = int(nx), int(ny)
        nbytes = state_bytes(self.desc)
        if nbytes == 0:
            # validation failed: surface the library's reason
            h = ctypes.c_void_p()
            check(lib.sclbm_bind(ctypes.byref(self.desc), None, 0, ctypes.byref(h)), "bind")
        self.nbytes = nbytes
        if buffer is None:
            buffer = torch.empty(nbytes, dtype=torch.uint8, device=device)
        assert buffer.numel() * buffer.element_size() >= nbytes and buffer.is_cuda
        self.buf = buffer
        self._h = ctypes.c_void_p()
        check(lib.sclbm_bind(ctypes.byref(self.desc), _dptr(self.buf), nbytes,
                             ctypes.byref(self._h)), "bind")
        if tiling == "auto":
            from . import autotune
            tiling = autotune.tiling_for(self.nx, self.ny, self.storage, self.boundary)
        if tiling is not None:
            self.set_tiling(*tiling)

    # ------------------------------------------------------------------ life
    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib.sclbm_release(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def storage(self) -> str:
        return {v: k for k, v in STORAGE.items()}[self.desc.storage]

    @property
    def boundary(self) -> str:
        return {v: k for k, v in BOUNDARY.items()}[self.desc.boundary]

    @property
    def handle(self):
        return self._h

    # ------------------------------------------------------------------ init
    def init_random(self, seed: int, mean=(0.7, 0.7), amp: float = 0.05, stream=None):
        m = (ctypes.c_double * 2)(*mean)
        check(lib.sclbm_init_random(self._h, ctypes.c_uint64(seed & (2 ** 64 - 1)), m,
                                    float(amp), _stream(stream)), "init_random")
        return self

    def init_fields(self, rho, ux=None, uy=None, stream=None):
        import torch
        dev = self.buf.device
        r = torch.as_tensor(np.ascontiguousarray(rho, dtype=np.float64)).to(dev)
        assert r.shape == (2, self.ny, self.nx)
        a, b = r[0].contiguous(), r[1].contiguous()
        vx = None if ux is None else torch.as_tensor(np.ascontiguousarray(ux, dtype=np.float64)).to(dev)
        vy = None if uy is None else torch.as_tensor(np.ascontiguousarray(uy, dtype=np.float64)).to(dev)
        check(lib.sclbm_init_fields(self._h, _dptr(a), _dptr(b), _dptr(vx), _dptr(vy),
                                    _stream(stream)), "init_fields")
        self._keep = (a, b, vx, vy)   # alive until the next call on this object
        return self

    # ------------------------------------------------------------------ run
    def step(self, n: int = 1, stream=None):
        check(lib.sclbm_step(self._h, int(n), _stream(stream)), "step")
        return self

    @property
    def t(self) -> int:
        v = ctypes.c_int64()
        check(lib.sclbm_time(self._h, ctypes.byref(v)), "time")
        return v.value

    def set_tiling(self, tile_x: int, tile_y: int, waves: int, stacked: int = 0,
                   throttle: int = 0, write_through: int = 0):
        t = Tiling(int(tile_x), int(tile_y), int(waves), int(stacked), int(throttle),
                   int(write_through))
        check(lib.sclbm_set_tiling(self._h, ctypes.byref(t)), "set_tiling")

    def get_tiling(self):
        t = Tiling()
        check(lib.sclbm_get_tiling(self._h, ctypes.byref(t)), "get_tiling")
        return (t.tile_x, t.tile_y, t.waves, t.stacked, t.throttle, t.write_through)

    # ------------------------------------------------------------------ read
    def moments_device(self, stream=None):
        """dict of (ny, nx) float64 CUDA tensors: rhoA, rhoB, ux, uy, sxy."""
        import torch
        out = {k: torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.buf.device)
               for k in ("rhoA", "rhoB", "ux", "uy", "sxy")}
        check(lib.sclbm_read_moments(self._h, *[_dptr(out[k]) for k in
                                               ("rhoA", "rhoB", "ux", "uy", "sxy")],
                                     _stream(stream)), "read_moments")
        return out

    def moments(self, stream=None) -> dict:
        d = self.moments_device(stream)
        return {k: v.cpu().numpy() for k, v in d.items()}

    def order_parameter(self, phi_ref=None, phi_out=None, stream=None):
        """(sum phi * phi_ref, sum phi^2) of phi = rho_A - rho_B now, in FP64;
        phi_ref / phi_out: float64 device tensors of shape (ny, nx) or None
        (phi_out receives phi)."""
        import torch
        for t in (phi_ref, phi_out):
            if t is not None:
                assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                assert tuple(t.shape) == (self.ny, self.nx)
        out = (ctypes.c_double * 2)()
        check(lib.sclbm_order_parameter(self._h, _dptr(phi_ref), _dptr(phi_out), out,
                                        _stream(stream)), "order_parameter")
        return float(out[0]), float(out[1])

    def diagnostics(self, stream=None, raise_nonfinite=False) -> dict:
        d = Diag()
        rc = lib.sclbm_diagnostics(self._h, ctypes.byref(d), _stream(stream))
        if rc != ENONFINITE or raise_nonfinite:
            check(rc, "diagnostics")
        return d.as_dict()

    def fused_diagnostics(self, stream=None) -> dict:
        d = Diag()
        rc = lib.sclbm_fused_diagnostics(self._h, ctypes.byref(d), _stream(stream))
        if rc != ENONFINITE:
            check(rc, "fused_diagnostics")
        return d.as_dict()

    def reset_wall_accum(self, stream=None):
        check(lib.sclbm_reset_wall_accum(self._h, _stream(stream)), "reset_wall_accum")

    # ------------------------------------------------------------ checkpoint
    def checkpoint(self, stream=None) -> bytes:
        n = lib.sclbm_checkpoint_bytes(self._h)
        buf = ctypes.create_string_buffer(n)
        check(lib.sclbm_checkpoint(self._h, buf, n, _stream(stream)), "checkpoint")
        return buf.raw

    def restore(self, data: bytes, stream=None):
        buf = ctypes.create_string_buffer(data, len(data))
        check(lib.sclbm_restore(self._h, buf, len(data), _stream(stream)), "restore")
        return self


def default_batch_tiling(nx: int, ny: int) -> tuple:
    """A 4-wave tiling usable inside a batch: stacked tiles for small
    lattices, 252-wide sweep strips otherwise."""
    if nx * ny <= (1 << 20):
        ns = -(-nx // 60)
        return (max(min(-(-nx // ns), 60), min(32, nx)), 4, 4, 1, 0)
    ns = -(-nx // 252)
    W = max(-(-nx // ns), min(32, nx))
    return (W, max(4, min(ny, 128)), 4, 0, 1)


class Batch:
    """Many Simulations (same storage) advanced together per `step` call:
    mode "persistent" runs each call as one cooperative launch with a grid
    barrier per step, "stepwise" as one ordinary launch per step covering
    every instance.  Each instance's result is bitwise equal to stepping it
    alone.  tilings: None (defaults), "auto" (tuned batch policy, which also
    picks the mode unless one is given) or a list of 5-tuples."""

    MODES = {"persistent": 0, "stepwise": 1}

    def __init__(self, sims, tilings=None, stream=None, mode=None):
        import torch
        self.sims = list(sims)
        n = len(self.sims)
        if tilings is None:
            tilings = [default_batch_tiling(s.nx, s.ny) for s in self.sims]
        elif isinstance(tilings, str):
            if tilings != "auto":
                raise ValueError("tilings: None, 'auto' or a list of 5-tuples")
            from . import autotune
            tilings, auto_mode = autotune.batch_plan(self.sims)
            mode = mode or auto_mode
        self.mode = mode or "persistent"
        if self.mode not in self.MODES:
            raise ValueError(f"mode must be one of {list(self.MODES)}")
        self.tilings = [tuple(t) for t in tilings]
        self._arr = (ctypes.c_void_p * n)(*[s.handle.value for s in self.sims])
        self._tl = (Tiling * n)(*[Tiling(*t) for t in self.tilings])
        nbytes = int(lib.sclbm_batch_bytes(self._arr, n, self._tl))
        if nbytes == 0:
            raise SclbmError(EINVAL, "batch_bytes")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.sims[0].buf.device)
        self._h = ctypes.c_void_p()
        check(lib.sclbm_batch_plan(self._arr, n, self._tl, _dptr(self.ws), nbytes,
                                   _stream(stream), ctypes.byref(self._h)), "batch_plan")
        check(lib.sclbm_batch_set_mode(self._h, self.MODES[self.mode]), "batch_set_mode")

    def step(self, steps, stream=None):
        n = len(self.sims)
        if isinstance(steps, int):
            steps = [steps] * n
        arr = (ctypes.c_int64 * n)(*[int(v) for v in steps])
        check(lib.sclbm_batch_step(self._h, arr, _stream(stream)), "batch_step")
        return self

    def status(self, stream=None):
        check(lib.sclbm_batch_status(self._h, _stream(stream)), "batch_status")

    def set_barrier_limit(self, sleeps: int = 0):
        """Sleeps a workgroup of the persistent mode waits at one grid barrier
        before the launch is reported failed (0: the default, seconds)."""
        check(lib.sclbm_batch_set_barrier_limit(self._h, int(sleeps)), "batch_set_barrier_limit")
        return self

    def info(self) -> dict:
        """capacity: co-resident workgroups of this kernel kind; tiles per
        step; kind (0 stacked, 1 sweep, 2 both); grid actually launched."""
        out = (ctypes.c_int32 * 3)()
        check(lib.sclbm_batch_info(self._h, out), "batch_info")
        return {"capacity": out[0], "tiles": out[1], "kind": out[2],
                "grid": min(out[0], out[1]) if self.mode == "persistent" else out[1],
                "mode": self.mode}

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib.sclbm_batch_release(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_step_static(sims, tilings=None, steps=1, stream=None):
    """Advance Simulations together as one STEPWISE batch without any device
    workspace: the batch tables go into the library's static device array
    (sclbm_batch_step_static).  Results equal Batch(..., mode="stepwise")."""
    sims = list(sims)
    n = len(sims)
    if tilings is None:
        tilings = [default_batch_tiling(s.nx, s.ny) for s in sims]
    if isinstance(steps, int):
        steps = [steps] * n
    arr = (ctypes.c_void_p * n)(*[s.handle.value for s in sims])
    tl = (Tiling * n)(*[Tiling(*t) for t in tilings])
    st = (ctypes.c_int64 * n)(*[int(v) for v in steps])
    check(lib.sclbm_batch_step_static(arr, n, tl, st, _stream(stream)), "batch_step_static")

