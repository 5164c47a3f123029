"""ctypes declarations of libtcm.so (include/tcm.h).  Marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtcm.so")

TCM_OK, TCM_E_ARG, TCM_E_CFL, TCM_E_POOL, TCM_E_RANGE, TCM_E_DEVICE, TCM_E_STATE, TCM_E_NOMEM = \
    0, -1, -2, -3, -4, -5, -6, -7
TCM_E_NONFINITE = -8
STATUS_NAMES = {0: "TCM_OK", -1: "TCM_E_ARG", -2: "TCM_E_CFL", -3: "TCM_E_POOL", -4: "TCM_E_RANGE",
                -5: "TCM_E_DEVICE", -6: "TCM_E_STATE", -7: "TCM_E_NOMEM", -8: "TCM_E_NONFINITE"}
MEDIA_DENSE, MEDIA_LAYERED, MEDIA_LATTICE = 0, 1, 2
ENGINE_BLOCKS, ENGINE_DENSE = 0, 1
FLAG_TIMING, FLAG_NO_GRAPH, FLAG_NO_UNIFORM_C2, FLAG_THREE_PASS_UPDATE, FLAG_DEBUG_CHECKS = 1, 2, 4, 8, 16
FLAG_C2_PLANES = 32

# every symbol include/tcm.h declares
EXPORTS = [
    "tcm_create", "tcm_create_batch", "tcm_add_source", "tcm_add_source_shot", "tcm_step",
    "tcm_read", "tcm_read_shot", "tcm_set_receivers", "tcm_read_traces", "tcm_adjoint",
    "tcm_reset", "tcm_stats", "tcm_destroy", "tcm_last_error", "tcm_version", "tcm_autotune", "tcm_autotune_run", "tcm_set_media",
    "tcm_set_launch", "tcm_snapshot", "tcm_restore", "tcm_snapshot_free", "tcm_hbm_probe",
    "tcm_read_noalloc", "tcm_check",
]


class Config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dt", C.c_double),
                ("trigger", C.c_float), ("retire", C.c_float),
                ("pool_bytes", C.c_uint64), ("device_pool", C.c_void_p), ("stream", C.c_void_p),
                ("engine", C.c_int32), ("flags", C.c_int32), ("checkpoint_every", C.c_int32),
                ("graph_steps", C.c_int32), ("wg_per_cu", C.c_int32),
                ("shutdown_steps", C.c_int32), ("shutdown_alpha", C.c_float),
                ("trigger_rel", C.c_float), ("retire_rel", C.c_float),
                ("trigger_interval", C.c_int32), ("blocks_per_wg", C.c_int32),
                ("blocks_per_wave", C.c_int32)]


class Media(C.Structure):
    _fields_ = [("kind", C.c_int32), ("c", C.c_void_p),
                ("nlayers", C.c_int32), ("z_top", C.c_void_p), ("c_layer", C.c_void_p),
                ("lattice", C.c_void_p), ("lx", C.c_int32), ("ly", C.c_int32), ("lz", C.c_int32),
                ("log2_spacing", C.c_int32)]


class Shot(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("media", Media)]


class Stats(C.Structure):
    _fields_ = [("step", C.c_int64), ("active_blocks", C.c_int64),
                ("peak_active_blocks", C.c_int64), ("pool_slots", C.c_int64),
                ("pool_bytes", C.c_int64), ("peak_pool_bytes", C.c_int64),
                ("table_bytes", C.c_int64), ("activations", C.c_int64),
                ("retirements", C.c_int64), ("cell_updates", C.c_int64),
                ("error", C.c_int32), ("nshots", C.c_int32),
                ("stencil_ms", C.c_double), ("stencil_launches", C.c_int64),
                ("stencil_cells", C.c_int64), ("uniform_cell_updates", C.c_int64),
                ("stencil_cells_uniform", C.c_int64), ("decay_block_steps", C.c_int64),
                ("trigger_level", C.c_double), ("retire_level", C.c_double),
                ("grad_cells", C.c_int64),
                ("adjoint_field_ms", C.c_double), ("adjoint_field_launches", C.c_int64),
                ("adjoint_field_cells", C.c_int64), ("adjoint_field_cells_uniform", C.c_int64),
                ("recompute_ms", C.c_double), ("recompute_launches", C.c_int64),
                ("recompute_cells", C.c_int64), ("recompute_cells_uniform", C.c_int64),
                ("checkpoint_bytes", C.c_int64), ("checkpoints", C.c_int64), ("adjoint_bytes", C.c_int64),
                ("lattice_cell_updates", C.c_int64), ("stencil_cells_lattice", C.c_int64),
                ("adjoint_field_cells_lattice", C.c_int64), ("recompute_cells_lattice", C.c_int64)]


class Tuning(C.Structure):
    _fields_ = [("wg_per_cu", C.c_int32), ("graph_steps", C.c_int32), ("ms_per_step", C.c_double),
                ("ncand", C.c_int32), ("cand_wg_per_cu", C.c_int32 * 32),
                ("cand_graph_steps", C.c_int32 * 32), ("cand_ms_per_step", C.c_double * 32),
                ("blocks_per_wg", C.c_int32), ("cand_blocks_per_wg", C.c_int32 * 32),
                ("blocks_per_wave", C.c_int32), ("cand_blocks_per_wave", C.c_int32 * 32),
                ("nfam", C.c_int32), ("fam_blocks_per_wg", C.c_int32 * 8), ("fam_blocks_per_wave", C.c_int32 * 8),
                ("fam_wg_per_cu", C.c_int32 * 8), ("fam_run_ms", C.c_double * 8)]


_lib = None


def lib():
    """Load libtcm.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1702_00216_amd.build` (hipcc, gfx950)")
        # PyTorch ships its own HIP runtime (same soname as /opt/rocm's).  Load it
        # first so that libtcm.so binds to that one copy: device pointers and
        # streams are then shared with torch, and only one runtime opens the GPU.
        try:
            import torch  # noqa: F401
            import torch.cuda  # noqa: F401
        except Exception:
            pass
        L = C.CDLL(LIB_PATH)
        P, I, F = C.c_void_p, C.c_int32, C.POINTER
        H = C.c_void_p
        L.tcm_create.argtypes = [F(Config), F(Media), F(H)]
        L.tcm_create_batch.argtypes = [F(Config), F(Shot), I, F(H)]
        L.tcm_add_source.argtypes = [H, I, I, I, P, I]
        L.tcm_add_source_shot.argtypes = [H, I, I, I, I, P, I]
        L.tcm_step.argtypes = [H, I]
        L.tcm_read.argtypes = [H, I, I, I, I, I, I, I, P, I]
        L.tcm_read_shot.argtypes = [H, I, I, I, I, I, I, I, I, P, I]
        L.tcm_read_noalloc.argtypes = [H, I, I, I, I, I, I, I, I, P]
        L.tcm_set_receivers.argtypes = [H, P, P, I]
        L.tcm_read_traces.argtypes = [H, P, I, F(C.c_int32)]
        L.tcm_adjoint.argtypes = [H, P, I, I, P, I]
        L.tcm_reset.argtypes = [H]
        L.tcm_snapshot.argtypes = [H, F(P)]
        L.tcm_restore.argtypes = [H, P]
        L.tcm_snapshot_free.argtypes = [P]
        L.tcm_snapshot_free.restype = None
        L.tcm_autotune.argtypes = [H, I, F(Tuning)]
        L.tcm_autotune_run.argtypes = [H, I, I, F(Tuning)]
        L.tcm_set_media.argtypes = [H, I, F(Media)]
        L.tcm_set_launch.argtypes = [H, I, I, I, I]
        L.tcm_hbm_probe.argtypes = [P, P, C.c_uint64, I, I, I, P, F(C.c_float)]
        L.tcm_stats.argtypes = [H, F(Stats)]
        L.tcm_check.argtypes = [H, F(C.c_int64)]
        L.tcm_destroy.argtypes = [H]
        L.tcm_destroy.restype = None
        L.tcm_last_error.argtypes = [H]
        L.tcm_last_error.restype = C.c_char_p
        L.tcm_version.argtypes = []
        L.tcm_version.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("tcm_destroy", "tcm_last_error", "tcm_version"):
                getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


class TCMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status
