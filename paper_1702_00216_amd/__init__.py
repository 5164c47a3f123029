"""Triggered Cells Method hot path on AMD Instinct MI355X (gfx950).

The compute path is libtcm.so (hand-written HIP kernels behind the C-ABI of
include/tcm.h); this package is its thin Python binding.  Importing it does
not touch the GPU; creating a :class:`Simulation` loads the library and fails
loudly if it has not been built.
"""
from ._lib import TCMError, EXPORTS, TCM_E_CFL, TCM_E_POOL, TCM_E_NONFINITE  # noqa: F401
from .sim import Simulation, Snapshot, hbm_probe, version  # noqa: F401

__all__ = ["Simulation", "TCMError", "version"]
