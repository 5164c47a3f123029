"""CPU oracle for the Triggered Cells Method hot path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it and
shares no code with it (the C sources here are compiled by gcc into their
own ``liboracle.so``).

What it computes (each function cites the passage it follows):

* :func:`dense_run`  -- O1, the leapfrog update of eq.(3) on the whole grid
  (zero field outside the domain), FP32 or FP64, with additive sources and
  receivers; ``ndim`` 1 or 2 selects the same central-difference operator in
  fewer dimensions (used by the closed-form pins).
* :class:`TCM`       -- O2, the Triggered Cells Method with the paper's cell
  bookkeeping (Table 1, "Boxes", "Time stepping", "Updating active cells").
* :func:`adjoint_f64` -- O3, the discrete adjoint of O1 in FP64.
* :func:`cfl_ok`, :func:`update_interval`, :func:`decay_total` -- eq.(4),
  eq.(5), eq.(6).

Parity of the paper's experiment figures (the 2000^3 / 4000^3 speed-up and
memory factors) is unpinned: their scenario and hardware are not given.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, "tcm_oracle.c"), os.path.join(_HERE, "tcm_oracle_impl.h")]

GCC_FLAGS = ["-O3", "-mavx2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
             "-shared", "-std=gnu11", "-Wall", "-Wno-unused-parameter"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", *GCC_FLAGS, "-o", tmp, _SRC[0], "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        _lib = C.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


_P = C.c_void_p
_I = C.c_int
_D = C.c_double
_I64P = C.POINTER(C.c_int64)


def _declare(L):
    for sfx in ("f32", "f64"):
        f = getattr(L, f"oracle_dense_{sfx}")
        f.argtypes = [_I, _I, _I, _I, _P, _D, _D, _P, _P, _I, _I,
                      _I, _P, _P, _P, _P, _P, _I, _P, _P]
        f.restype = _I
        f = getattr(L, f"otcm_create_{sfx}")
        real = C.c_float if sfx == "f32" else C.c_double
        f.argtypes = [_I, _I, _I, _I, _P, _D, _D, real, real, _I]
        f.restype = _P
        getattr(L, f"otcm_destroy_{sfx}").argtypes = [_P]
        getattr(L, f"otcm_destroy_{sfx}").restype = None
        f = getattr(L, f"otcm_add_source_{sfx}")
        f.argtypes = [_P, _I, _I, _I, _P, _I]
        f.restype = _I
        f = getattr(L, f"otcm_set_receivers_{sfx}")
        f.argtypes = [_P, _P, _I]
        f.restype = _I
        f = getattr(L, f"otcm_step_{sfx}")
        f.argtypes = [_P, _I, _P, C.c_uint]
        f.restype = _I
        for name in ("otcm_read", "otcm_stats", "otcm_triggered"):
            f = getattr(L, f"{name}_{sfx}")
            f.argtypes = [_P, _I, _P] if name == "otcm_read" else [_P, _P]
            f.restype = _I
        f = getattr(L, f"otcm_check_{sfx}")
        f.argtypes = [_P]
        f.restype = _I
        f = getattr(L, f"otcm_set_shutdown_{sfx}")
        f.argtypes = [_P, _I, real]
        f.restype = _I
        f = getattr(L, f"otcm_set_adaptive_{sfx}")
        f.argtypes = [_P, real, real]
        f.restype = _I
        f = getattr(L, f"otcm_levels_{sfx}")
        f.argtypes = [_P, _P]
        f.restype = _I
        f = getattr(L, f"otcm_set_interval_{sfx}")
        f.argtypes = [_P, _I]
        f.restype = _I
    L.oracle_adjoint_f64.argtypes = [_I, _I, _I, _P, _D, _D, _I, _P, _P, _P, _P, _P,
                                     _I, _P, _I, _P, _I, _P]
    L.oracle_adjoint_f64.restype = _I
    L.oracle_cfl_ok.argtypes = [_D, _D, _D, _I]
    L.oracle_cfl_ok.restype = _I
    L.oracle_update_interval.argtypes = [_D, _D, _D, _D]
    L.oracle_update_interval.restype = _D
    L.oracle_decay_total.argtypes = [_D, _I]
    L.oracle_decay_total.restype = _D
    L.oracle_openmp_threads.argtypes = []
    L.oracle_openmp_threads.restype = _I
    L.oracle_set_threads.argtypes = [_I]
    L.oracle_set_threads.restype = None
    L.oracle_stream_triad.argtypes = [C.c_long, _I]
    L.oracle_stream_triad.restype = _D


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_P)


def _dt(dtype) -> Tuple[np.dtype, str]:
    dtype = np.dtype(dtype)
    if dtype == np.float32:
        return dtype, "f32"
    if dtype == np.float64:
        return dtype, "f64"
    raise ValueError("dtype must be float32 or float64")


class Sources:
    """Flattened point-source table: linear cell index, start step, samples."""

    def __init__(self, shape, sources: Sequence, dtype):
        nx, ny, nz = shape
        idx, t0, ns, off, ws = [], [], [], [], []
        o = 0
        for src in sources:
            (x, y, z), w = src[0], np.asarray(src[1])
            start = int(src[2]) if len(src) > 2 else 0
            if not (0 <= x < nx and 0 <= y < ny and 0 <= z < nz):
                raise ValueError("source outside the domain")
            idx.append(x + nx * (y + ny * z))
            t0.append(start)
            ns.append(w.size)
            off.append(o)
            ws.append(w.astype(dtype))
            o += w.size
        self.n = len(idx)
        self.idx = np.array(idx or [0], np.int64)
        self.t0 = np.array(t0 or [0], np.int32)
        self.ns = np.array(ns or [0], np.int32)
        self.off = np.array(off or [0], np.int64)
        self.w = np.concatenate(ws) if ws else np.zeros(1, dtype)


def _rec_idx(shape, receivers) -> np.ndarray:
    nx, ny, nz = shape
    if receivers is None or len(receivers) == 0:
        return np.zeros(1, np.int64)
    r = np.asarray(receivers, np.int64).reshape(-1, 3)
    if np.any(r < 0) or np.any(r[:, 0] >= nx) or np.any(r[:, 1] >= ny) or np.any(r[:, 2] >= nz):
        raise ValueError("receiver outside the domain")
    return r[:, 0] + nx * (r[:, 1] + ny * r[:, 2])


def dense_run(c: np.ndarray, dt: float, dx: float, steps: int, dtype=np.float32,
              phi: Optional[np.ndarray] = None, phi_prev: Optional[np.ndarray] = None,
              step0: int = 0, sources: Sequence = (), receivers=None, ndim: int = 3):
    """O1: ``steps`` leapfrog steps of eq.(3) on the whole grid.

    ``c`` is (nz, ny, nx) (x fastest).  ``sources`` is a sequence of
    ``((x, y, z), w)`` or ``((x, y, z), w, start_step)``; sample k is added to
    phi^{n+1} at the source cell in step n = start + k.  Returns
    ``(phi^n, phi^{n-1}, traces)`` with traces[i, r] = phi^{step0+i+1} at
    receiver r.
    """
    dtype, sfx = _dt(dtype)
    c = np.ascontiguousarray(c, dtype=dtype)
    nz, ny, nx = c.shape
    phi = np.zeros_like(c) if phi is None else np.array(phi, dtype=dtype, copy=True, order="C")
    phi_prev = np.zeros_like(c) if phi_prev is None else np.array(phi_prev, dtype=dtype, copy=True, order="C")
    src = Sources((nx, ny, nz), sources, dtype)
    ridx = _rec_idx((nx, ny, nz), receivers)
    nrec = 0 if receivers is None else len(ridx)
    traces = np.zeros((max(steps, 1), max(nrec, 1)), dtype)
    rc = getattr(lib(), f"oracle_dense_{sfx}")(
        nx, ny, nz, ndim, _ptr(c), dt, dx, _ptr(phi), _ptr(phi_prev), step0, steps,
        src.n, _ptr(src.idx), _ptr(src.t0), _ptr(src.ns), _ptr(src.off), _ptr(src.w),
        nrec, _ptr(ridx), _ptr(traces))
    if rc != 0:
        raise RuntimeError(f"oracle_dense failed: {rc}")
    return phi, phi_prev, traces[:steps, :nrec]


class TCM:
    """O2: CPU Triggered Cells Method (paper's cell/box bookkeeping).

    ``block`` is the cell edge in nodes (8 on the hot path), ``trigger`` and
    ``retire`` are absolute |phi| levels, ``cap`` the maximum number of boxes
    (0: one per cell).  ``step`` returns 0, or -3 when the cap is exceeded.
    """

    E_POOL = -3

    def __init__(self, c: np.ndarray, dt: float, dx: float, trigger: float = 0.0,
                 retire: float = 0.0, block: int = 8, cap: int = 0, dtype=np.float32,
                 shutdown_steps: int = 0, shutdown_alpha: float = 1.0,
                 trigger_rel: float = 0.0, retire_rel: float = 0.0, interval: int = 1):
        self.dtype, self.sfx = _dt(dtype)
        c = np.ascontiguousarray(c, dtype=self.dtype)
        self.shape = (c.shape[2], c.shape[1], c.shape[0])
        self.block = block
        L = lib()
        self._h = getattr(L, f"otcm_create_{self.sfx}")(
            self.shape[0], self.shape[1], self.shape[2], block, _ptr(c), dt, dx,
            trigger, retire, cap)
        if not self._h:
            raise MemoryError("otcm_create failed")
        self.nrec = 0
        if shutdown_steps:
            if self._f("otcm_set_shutdown")(self._h, int(shutdown_steps), shutdown_alpha) != 0:
                raise ValueError("shutdown_steps must be in [0, 255]")
        if interval != 1:
            if self._f("otcm_set_interval")(self._h, int(interval)) != 0:
                raise ValueError("interval must be in [1, block edge]")
        if trigger_rel or retire_rel:
            if self._f("otcm_set_adaptive")(self._h, trigger_rel, retire_rel) != 0:
                raise ValueError("need 0 <= retire_rel <= trigger_rel")
        nx, ny, nz = self.shape
        self.cells_shape = (-(-nz // block), -(-ny // block), -(-nx // block))

    def _f(self, name):
        return getattr(lib(), f"{name}_{self.sfx}")

    def close(self):
        if self._h:
            self._f("otcm_destroy")(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_source(self, xyz, w) -> int:
        w = np.ascontiguousarray(w, dtype=self.dtype)
        return self._f("otcm_add_source")(self._h, int(xyz[0]), int(xyz[1]), int(xyz[2]),
                                          _ptr(w), int(w.size))

    def set_receivers(self, rec) -> int:
        r = np.ascontiguousarray(np.asarray(rec, np.int32).reshape(-1, 3))
        self.nrec = r.shape[0]
        return self._f("otcm_set_receivers")(self._h, _ptr(r), self.nrec)

    def step(self, n: int, order_seed: int = 0, traces: bool = False):
        tr = np.zeros((max(n, 1), max(self.nrec, 1)), self.dtype) if traces else None
        rc = self._f("otcm_step")(self._h, n, _ptr(tr), order_seed)
        if traces:
            return rc, tr[:n, :self.nrec]
        return rc

    def read(self, which: int = 0) -> np.ndarray:
        nx, ny, nz = self.shape
        out = np.empty((nz, ny, nx), self.dtype)
        self._f("otcm_read")(self._h, which, _ptr(out))
        return out

    def stats(self) -> dict:
        s = np.zeros(8, np.int64)
        self._f("otcm_stats")(self._h, _ptr(s))
        keys = ["step", "active", "peak_active", "boxes", "activations", "retirements",
                "updates", "error"]
        return dict(zip(keys, (int(v) for v in s)))

    def triggered(self) -> np.ndarray:
        out = np.zeros(self.cells_shape, np.uint8)
        self._f("otcm_triggered")(self._h, _ptr(out))
        return out

    def levels(self):
        """(trigger, keep level) used by the last activation update."""
        out = np.zeros(2, self.dtype)
        self._f("otcm_levels")(self._h, _ptr(out))
        return float(out[0]), float(out[1])

    def check(self) -> int:
        return self._f("otcm_check")(self._h)


def adjoint_f64(c: np.ndarray, dt: float, dx: float, sources: Sequence, receivers,
                resid: np.ndarray, ckpt: int = 50) -> np.ndarray:
    """O3: dJ/dc (FP64) for traces[n, r] = u^{n+1}[rec r] and dJ/dtraces = resid."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    nz, ny, nx = c.shape
    src = Sources((nx, ny, nz), sources, np.float64)
    ridx = _rec_idx((nx, ny, nz), receivers)
    resid = np.ascontiguousarray(resid, dtype=np.float64)
    nt = resid.shape[0]
    assert resid.shape[1] == len(ridx)
    grad = np.zeros_like(c)
    rc = lib().oracle_adjoint_f64(nx, ny, nz, _ptr(c), dt, dx, src.n, _ptr(src.idx),
                                  _ptr(src.t0), _ptr(src.ns), _ptr(src.off), _ptr(src.w),
                                  len(ridx), _ptr(ridx), nt, _ptr(resid), ckpt, _ptr(grad))
    if rc != 0:
        raise RuntimeError(f"oracle_adjoint_f64 failed: {rc}")
    return grad


def cfl_ok(cmax: float, dt: float, dx: float, ndim: int = 3) -> bool:
    """eq.(4) with equal spacing: (c dt / dx)^2 * ndim <= 1."""
    return bool(lib().oracle_cfl_ok(cmax, dt, dx, ndim))


def update_interval(dx: float, cell_len: float, c: float, dt: float) -> float:
    """eq.(5): n = dx * L_cell / (2 c dt)."""
    return float(lib().oracle_update_interval(dx, cell_len, c, dt))


def decay_total(alpha: float, n: int) -> float:
    """eq.(6): A = alpha^n."""
    return float(lib().oracle_decay_total(alpha, n))


def openmp_threads() -> int:
    return int(lib().oracle_openmp_threads())


def stream_triad(n: int = 1 << 26, reps: int = 5) -> float:
    """Host STREAM triad bandwidth in GB/s with the current thread count."""
    return float(lib().oracle_stream_triad(int(n), int(reps)))


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's parallel loops from now on."""
    lib().oracle_set_threads(int(n))
