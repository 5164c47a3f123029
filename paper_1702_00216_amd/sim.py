"""Python front end of libtcm.so: argument marshalling only.

Every step of the method runs in the HIP kernels behind the C-ABI; this
module converts NumPy / torch arguments to pointers and sizes.  Torch is used
for device memory (reads into device tensors) and streams.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np

from . import _lib as L


def _media_struct(media, shape, keep: list) -> L.Media:
    """Accepts a float32 (nz, ny, nx) array, or an object with z_top/c_layer
    (layered) or lattice/spacing (lattice)."""
    m = L.Media()
    if isinstance(media, np.ndarray):
        c = np.ascontiguousarray(media, dtype=np.float32)
        nx, ny, nz = shape
        if c.shape != (nz, ny, nx):
            raise ValueError(f"dense media must have shape (nz, ny, nx) = {(nz, ny, nx)}")
        keep.append(c)
        m.kind = L.MEDIA_DENSE
        m.c = c.ctypes.data
    elif hasattr(media, "z_top"):
        zt = np.ascontiguousarray(media.z_top, dtype=np.int32)
        cl = np.ascontiguousarray(media.c_layer, dtype=np.float32)
        keep += [zt, cl]
        m.kind = L.MEDIA_LAYERED
        m.nlayers = zt.size
        m.z_top = zt.ctypes.data
        m.c_layer = cl.ctypes.data
    elif hasattr(media, "lattice"):
        lat = np.ascontiguousarray(media.lattice, dtype=np.float64)
        keep.append(lat)
        s = int(media.spacing)
        if s <= 0 or s & (s - 1):
            raise ValueError("lattice spacing must be a power of two")
        m.kind = L.MEDIA_LATTICE
        m.lattice = lat.ctypes.data
        m.lz, m.ly, m.lx = lat.shape
        m.log2_spacing = s.bit_length() - 1
    else:
        raise TypeError("unsupported media description")
    return m


class Simulation:
    """One TCM handle (single shot or a batch of shots over one pool).

    ``shape`` is (nx, ny, nz) (or a list of shapes with ``media`` a list, for a
    batch); ``engine`` "blocks" runs the TCM, "dense" updates every node.
    """

    def __init__(self, shape, dx: float, dt: float, media, trigger: float = 0.0,
                 retire: float = 0.0, pool_bytes: int = 0, engine: str = "blocks",
                 timing: bool = False, graphs: bool = True, stream=None,
                 checkpoint_every: int = 0, graph_steps: int = 0, wg_per_cu: int = 0,
                 device_pool=None, uniform_c2: bool = True, shutdown_steps: int = 0,
                 shutdown_alpha: float = 1.0, trigger_rel: float = 0.0, retire_rel: float = 0.0,
                 trigger_interval: int = 1, blocks_per_wg: int = 0, blocks_per_wave: int = 0,
                 three_pass_update: bool = False, debug_checks: bool = False,
                 c2_planes: bool = False):
        lib = L.lib()
        cfg = L.Config()
        cfg.dx, cfg.dt = float(dx), float(dt)
        cfg.trigger, cfg.retire = float(trigger), float(retire)
        cfg.pool_bytes = int(pool_bytes)
        cfg.engine = L.ENGINE_DENSE if engine == "dense" else L.ENGINE_BLOCKS
        cfg.flags = ((L.FLAG_TIMING if timing else 0) | (0 if graphs else L.FLAG_NO_GRAPH)
                     | (0 if uniform_c2 else L.FLAG_NO_UNIFORM_C2)
                     | (L.FLAG_THREE_PASS_UPDATE if three_pass_update else 0)
                     | (L.FLAG_DEBUG_CHECKS if debug_checks else 0)
                     | (L.FLAG_C2_PLANES if c2_planes else 0))
        cfg.checkpoint_every = int(checkpoint_every)
        cfg.graph_steps = int(graph_steps)
        cfg.wg_per_cu = int(wg_per_cu)
        cfg.shutdown_steps = int(shutdown_steps)
        cfg.shutdown_alpha = float(shutdown_alpha)
        cfg.trigger_rel = float(trigger_rel)
        cfg.retire_rel = float(retire_rel)
        cfg.trigger_interval = int(trigger_interval)
        cfg.blocks_per_wg = int(blocks_per_wg)
        cfg.blocks_per_wave = int(blocks_per_wave)
        self._pool_tensor = device_pool
        if device_pool is not None:
            cfg.device_pool = device_pool.data_ptr()
        if stream is not None:
            cfg.stream = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        self._stream = stream
        keep: list = []
        h = C.c_void_p()
        batch = isinstance(shape, (list, tuple)) and len(shape) > 0 and isinstance(shape[0], (list, tuple))
        if batch:
            if len(shape) != len(media):
                raise ValueError("one media per shot")
            shots = (L.Shot * len(shape))()
            for i, (shp, med) in enumerate(zip(shape, media)):
                shots[i].nx, shots[i].ny, shots[i].nz = (int(v) for v in shp)
                shots[i].media = _media_struct(med, tuple(int(v) for v in shp), keep)
            rc = lib.tcm_create_batch(C.byref(cfg), shots, len(shape), C.byref(h))
            self.shapes = [tuple(int(v) for v in s) for s in shape]
        else:
            cfg.nx, cfg.ny, cfg.nz = (int(v) for v in shape)
            m = _media_struct(media, tuple(int(v) for v in shape), keep)
            rc = lib.tcm_create(C.byref(cfg), C.byref(m), C.byref(h))
            self.shapes = [tuple(int(v) for v in shape)]
        if rc != 0:
            raise L.TCMError(rc, lib.tcm_last_error(None).decode())
        self._h = h
        self.shape = self.shapes[0]
        self.nrec = 0

    # ------------------------------------------------------------------
    def _check(self, rc: int):
        if rc != 0:
            raise L.TCMError(rc, L.lib().tcm_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            L.lib().tcm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------------
    def add_source(self, xyz, w, shot: int = 0):
        w = np.ascontiguousarray(w, dtype=np.float32)
        self._check(L.lib().tcm_add_source_shot(self._h, shot, int(xyz[0]), int(xyz[1]), int(xyz[2]),
                                                w.ctypes.data, w.size))

    def set_receivers(self, rec, shots: Optional[Sequence[int]] = None):
        r = np.ascontiguousarray(np.asarray(rec, dtype=np.int32).reshape(-1, 3))
        s = None if shots is None else np.ascontiguousarray(shots, dtype=np.int32)
        self.nrec = r.shape[0]
        self._check(L.lib().tcm_set_receivers(self._h, r.ctypes.data,
                                              None if s is None else s.ctypes.data, self.nrec))

    def step(self, n: int):
        """Advance n steps; raises TCMError (TCM_E_POOL) if the pool overflowed,
        (TCM_E_NONFINITE) if a step wrote a NaN or infinite value."""
        self._check(L.lib().tcm_step(self._h, int(n)))

    def step_status(self, n: int) -> int:
        return int(L.lib().tcm_step(self._h, int(n)))

    def last_error(self) -> str:
        """Message of the handle's last failed call."""
        return L.lib().tcm_last_error(self._h).decode()

    def read(self, which: int = 0, box=None, shot: int = 0, out=None) -> np.ndarray:
        """phi^n (which=0) or phi^{n-1} (which=1) of a box ((x0,y0,z0),(sx,sy,sz))
        as a float32 (sz, sy, sx) array, or into ``out`` (a CUDA torch tensor)."""
        nx, ny, nz = self.shapes[shot]
        (x0, y0, z0), (sx, sy, sz) = box if box is not None else ((0, 0, 0), (nx, ny, nz))
        if out is not None:
            import torch
            if not (out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
                    and out.numel() == sx * sy * sz):
                raise ValueError("out must be a contiguous float32 CUDA tensor of the box size")
            torch.cuda.current_stream().synchronize()
            self._check(L.lib().tcm_read_shot(self._h, shot, which, x0, y0, z0, sx, sy, sz,
                                              out.data_ptr(), 1))
            self._check(L.lib().tcm_stats(self._h, C.byref(L.Stats())))   # orders the read
            return out
        a = np.empty((sz, sy, sx), np.float32)
        self._check(L.lib().tcm_read_shot(self._h, shot, which, x0, y0, z0, sx, sy, sz,
                                          a.ctypes.data, 0))
        return a

    def read_traces(self) -> np.ndarray:
        n = C.c_int32(0)
        self._check(L.lib().tcm_read_traces(self._h, None, 0, C.byref(n)))
        out = np.zeros((n.value, self.nrec), np.float32)
        if n.value and self.nrec:
            self._check(L.lib().tcm_read_traces(self._h, out.ctypes.data, 0, C.byref(n)))
        return out

    def adjoint(self, resid: np.ndarray) -> np.ndarray:
        r = np.ascontiguousarray(resid, dtype=np.float32)
        nx, ny, nz = self.shape
        g = np.zeros((nz, ny, nx), np.float32)
        self._check(L.lib().tcm_adjoint(self._h, r.ctypes.data, r.shape[0], 0, g.ctypes.data, 0))
        return g

    def adjoint_device(self, resid, grad):
        """resid and grad are contiguous float32 CUDA tensors ([nt, nrec], [nz, ny, nx])."""
        import torch
        torch.cuda.current_stream().synchronize()
        self._check(L.lib().tcm_adjoint(self._h, resid.data_ptr(), resid.shape[0], 1,
                                        grad.data_ptr(), 1))
        return grad

    def autotune(self, probe_steps: int = 32, cache: Optional[str] = None,
                 key: Optional[str] = None) -> dict:
        """Pick the launch shape (stencil workgroup tile of 2, 4 or 8 blocks,
        one or two blocks per wave, workgroups per CU, steps per graph) by
        timing probe_steps steps from
        the current state for each candidate; the state is unchanged.  With
        ``cache`` (a JSON file) and ``key``, a stored choice is applied
        without probing and new choices are stored."""
        import json
        import os
        if cache and key and os.path.exists(cache):
            with open(cache) as f:
                stored = json.load(f).get(key)
            if stored and "blocks_per_wave" in stored:
                self._apply_tuning(stored["wg_per_cu"], stored["graph_steps"], stored["blocks_per_wg"],
                                   stored["blocks_per_wave"])
                return dict(stored, cached=True)
        t = L.Tuning()
        self._check(L.lib().tcm_autotune(self._h, int(probe_steps), C.byref(t)))
        res = {"blocks_per_wg": t.blocks_per_wg, "blocks_per_wave": t.blocks_per_wave,
               "wg_per_cu": t.wg_per_cu, "graph_steps": t.graph_steps, "ms_per_step": t.ms_per_step,
               "cached": False,
               "candidates": [(t.cand_blocks_per_wg[i], t.cand_blocks_per_wave[i], t.cand_wg_per_cu[i],
                               t.cand_graph_steps[i], t.cand_ms_per_step[i]) for i in range(t.ncand)]}
        if cache and key:
            data = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    data = json.load(f)
            data[key] = {k: res[k] for k in ("blocks_per_wg", "blocks_per_wave", "wg_per_cu", "graph_steps",
                                             "ms_per_step")}
            with open(cache, "w") as f:
                json.dump(data, f, indent=1)
        return res

    def autotune_run(self, nsteps: int, probe_steps: int = 32, cache: Optional[str] = None,
                     key: Optional[str] = None) -> dict:
        """Pick the launch shape for a run of ``nsteps`` steps from the current
        state (tcm_autotune_run): candidates probed at three states along the
        run, then each tile family's best timed over the whole run; the state
        is unchanged.  ``cache`` / ``key`` as for :meth:`autotune`."""
        import json
        import os
        if cache and key and os.path.exists(cache):
            with open(cache) as f:
                stored = json.load(f).get(key)
            if stored and "families" in stored:
                self._apply_tuning(stored["wg_per_cu"], stored["graph_steps"], stored["blocks_per_wg"],
                                   stored["blocks_per_wave"])
                return dict(stored, cached=True)
        t = L.Tuning()
        self._check(L.lib().tcm_autotune_run(self._h, int(nsteps), int(probe_steps), C.byref(t)))
        res = {"blocks_per_wg": t.blocks_per_wg, "blocks_per_wave": t.blocks_per_wave,
               "wg_per_cu": t.wg_per_cu, "graph_steps": t.graph_steps, "ms_per_step": t.ms_per_step,
               "cached": False,
               "families": {f"{t.fam_blocks_per_wg[i]}x{t.fam_blocks_per_wave[i]}@{t.fam_wg_per_cu[i]}":
                            round(t.fam_run_ms[i], 3) for i in range(t.nfam)},
               "candidates": [(t.cand_blocks_per_wg[i], t.cand_blocks_per_wave[i], t.cand_wg_per_cu[i],
                               t.cand_graph_steps[i], t.cand_ms_per_step[i]) for i in range(t.ncand)]}
        if cache and key:
            data = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    data = json.load(f)
            data[key] = {k: res[k] for k in ("blocks_per_wg", "blocks_per_wave", "wg_per_cu", "graph_steps",
                                             "ms_per_step", "families")}
            with open(cache, "w") as f:
                json.dump(data, f, indent=1)
        return res

    def _apply_tuning(self, wg_per_cu: int, graph_steps: int, blocks_per_wg: int = 0,
                      blocks_per_wave: int = 0):
        self._check(L.lib().tcm_set_launch(self._h, int(wg_per_cu), int(graph_steps), int(blocks_per_wg),
                                           int(blocks_per_wave)))

    def set_launch(self, wg_per_cu: int, graph_steps: int, blocks_per_wg: int = 0,
                   blocks_per_wave: int = 0):
        """Launch shape: workgroups per CU, steps per graph, workgroup tile
        (2, 4 or 8 blocks) and blocks per wave (1 or 2); 0 keeps the current
        tile or blocks per wave."""
        self._apply_tuning(wg_per_cu, graph_steps, blocks_per_wg, blocks_per_wave)

    def reset(self):
        self._check(L.lib().tcm_reset(self._h))
        self.nrec = 0

    def set_media(self, media, shot: int = 0):
        """New wave speed for a shot (same kind and sizes as at creation); the
        handle returns to level 0 as after :meth:`reset` (tcm_set_media)."""
        keep: list = []
        m = _media_struct(media, self.shapes[shot], keep)
        self._check(L.lib().tcm_set_media(self._h, int(shot), C.byref(m)))
        self.nrec = 0

    def snapshot(self) -> "Snapshot":
        """Device copy of the whole state at the current step (tcm_snapshot)."""
        p = C.c_void_p()
        self._check(L.lib().tcm_snapshot(self._h, C.byref(p)))
        return Snapshot(p, self)

    def restore(self, snap: "Snapshot"):
        """Return to the step and state of ``snap`` (taken from this handle)."""
        self._check(L.lib().tcm_restore(self._h, snap._p))

    def check(self) -> int:
        """Violations of the block-table invariants (tcm_check); 0 when consistent."""
        v = C.c_int64(0)
        self._check(L.lib().tcm_check(self._h, C.byref(v)))
        return int(v.value)

    def stats(self) -> dict:
        s = L.Stats()
        self._check(L.lib().tcm_stats(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in L.Stats._fields_}


class Snapshot:
    """A state saved by Simulation.snapshot(); frees its device memory when
    garbage-collected or closed (before its handle is destroyed)."""

    def __init__(self, p, owner):
        self._p = p
        self._owner = owner          # keeps the handle alive while the snapshot lives

    def close(self):
        if getattr(self, "_p", None):
            L.lib().tcm_snapshot_free(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def version() -> str:
    return L.lib().tcm_version().decode()


def hbm_probe(nread: int = 3, n: int = 1 << 28, wg_per_cu: int = 0, reps: int = 5) -> dict:
    """Achievable HBM bandwidth of a plain streaming kernel in the fastest
    shape measured (tcm_hbm_probe): nread sources of n floats each (n a
    multiple of 4096), one destination.
    Returns the best launch time and the GB/s it moves."""
    import torch
    src = torch.ones(nread * n, dtype=torch.float32, device="cuda")
    dst = torch.empty(n, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    ms = C.c_float(0.0)
    rc = L.lib().tcm_hbm_probe(src.data_ptr(), dst.data_ptr(), n, nread, wg_per_cu, reps, stream,
                               C.byref(ms))
    if rc != 0:
        raise L.TCMError(rc, L.lib().tcm_last_error(None).decode())
    ok = bool(torch.all(dst == float(nread)).item())
    del src, dst
    nbytes = (nread + 1) * 4 * n
    return {"nread": nread, "bytes": nbytes, "best_ms": ms.value,
            "GBps": nbytes / (ms.value * 1e-3) / 1e9, "wg_per_cu": wg_per_cu or 8, "result_ok": ok}
