"""Host-side checks of libtcm.so that need no GPU: the library loads, exports
every symbol include/tcm.h declares, and rejects invalid problems (eq.(4),
media, thresholds) before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from conftest import ROOT

pa = pytest.importorskip("paper_1702_00216_amd")
from paper_1702_00216_amd import _lib as L  # noqa: E402


def _declared():
    src = open(os.path.join(ROOT, "include", "tcm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tcm_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    names = _declared()
    assert set(names) == set(L.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n
    assert b"gfx950" in lib.tcm_version()


def _create(shape, c, dt, dx=1.0, trigger=0.0, retire=0.0, **kw):
    cfg = L.Config()
    cfg.nx, cfg.ny, cfg.nz = shape
    cfg.dx, cfg.dt = dx, dt
    cfg.trigger, cfg.retire = trigger, retire
    for k, v in kw.items():
        setattr(cfg, k, v)
    m = L.Media()
    m.kind = L.MEDIA_DENSE
    m.c = c.ctypes.data
    h = C.c_void_p()
    rc = L.lib().tcm_create(C.byref(cfg), C.byref(m), C.byref(h))
    if rc == 0:
        L.lib().tcm_destroy(h)
    return rc, L.lib().tcm_last_error(None).decode()


def test_cfl_violation_rejected():
    c = np.ones((4, 4, 4), np.float32)
    rc, msg = _create((4, 4, 4), c, dt=0.58)          # 0.58 > 1/sqrt(3)
    assert rc == L.TCM_E_CFL and "eq.(4)" in msg
    c[2, 2, 2] = 2.0
    rc, _ = _create((4, 4, 4), c, dt=0.3)             # max c decides
    assert rc == L.TCM_E_CFL


@pytest.mark.parametrize("bad", [-1.0, np.nan, np.inf])
def test_bad_speed_rejected(bad):
    c = np.ones((4, 4, 4), np.float32)
    c[1, 2, 3] = bad
    rc, msg = _create((4, 4, 4), c, dt=0.5)
    assert rc == L.TCM_E_ARG and "node" in msg


def test_bad_thresholds_rejected():
    c = np.ones((4, 4, 4), np.float32)
    assert _create((4, 4, 4), c, 0.5, trigger=1e-7, retire=1e-6)[0] == L.TCM_E_ARG
    assert _create((4, 4, 4), c, 0.5, trigger=-1.0, retire=-1.0)[0] == L.TCM_E_ARG
    assert _create((4, 4, 4), c, 0.5, dx=0.0)[0] == L.TCM_E_ARG


def test_bad_configuration_rejected():
    c = np.ones((4, 4, 4), np.float32)
    assert _create((4, 4, 4), c, 0.5, blocks_per_wg=3)[0] == L.TCM_E_ARG
    assert _create((4, 4, 4), c, 0.5, blocks_per_wave=3)[0] == L.TCM_E_ARG
    assert _create((4, 4, 4), c, 0.5, blocks_per_wg=2, blocks_per_wave=2)[0] == L.TCM_E_ARG
    assert _create((4, 4, 4), c, 0.5, trigger_interval=9)[0] == L.TCM_E_ARG
    assert _create((4, 4, 4), c, 0.5, shutdown_steps=300, shutdown_alpha=0.5)[0] == L.TCM_E_ARG
    assert _create((4, 4, 4), c, 0.5, trigger_rel=1e-4, retire_rel=1e-3)[0] == L.TCM_E_ARG
    rc, msg = _create((4, 4, 4), c, 0.5, device_pool=1234)
    assert rc == L.TCM_E_ARG and "pool_bytes" in msg


def test_lattice_media_validated():
    cfg = L.Config()
    cfg.nx = cfg.ny = cfg.nz = 64
    cfg.dx, cfg.dt = 1.0, 0.5 / 4500
    lat = np.full((4, 4, 4), 3000.0)
    m = L.Media()
    m.kind = L.MEDIA_LATTICE
    m.lattice = lat.ctypes.data
    m.lx = m.ly = m.lz = 4
    m.log2_spacing = 4          # needs (63 >> 4) + 2 = 5 nodes per axis
    h = C.c_void_p()
    assert L.lib().tcm_create(C.byref(cfg), C.byref(m), C.byref(h)) == L.TCM_E_ARG
    assert "lattice" in L.lib().tcm_last_error(None).decode()


def test_simulation_without_device_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(pa.TCMError):
        pa.Simulation((16, 16, 16), 1.0, 0.5, np.ones((16, 16, 16), np.float32))


def test_hbm_probe_arguments_validated():
    """tcm_hbm_probe rejects bad arguments before any device call (the
    pointers below are never dereferenced)."""
    lib = L.lib()
    ms = C.c_float(0.0)
    src, dst = 1 << 20, 1 << 40
    assert lib.tcm_hbm_probe(None, dst, 4096, 3, 0, 1, None, C.byref(ms)) == L.TCM_E_ARG
    assert lib.tcm_hbm_probe(src, dst, 4096, 3, 0, 1, None, None) == L.TCM_E_ARG
    assert lib.tcm_hbm_probe(src, dst, 0, 3, 0, 1, None, C.byref(ms)) == L.TCM_E_ARG
    assert lib.tcm_hbm_probe(src, dst, 3000, 3, 0, 1, None, C.byref(ms)) == L.TCM_E_ARG
    assert "multiple of 4096" in lib.tcm_last_error(None).decode()
    assert lib.tcm_hbm_probe(src, dst, 4096, 4, 0, 1, None, C.byref(ms)) == L.TCM_E_ARG
    assert lib.tcm_hbm_probe(src, dst, 4096, 3, 33, 1, None, C.byref(ms)) == L.TCM_E_ARG
    assert lib.tcm_hbm_probe(src, dst, 4096, 3, 0, 0, None, C.byref(ms)) == L.TCM_E_ARG
    assert lib.tcm_hbm_probe(src + 4, dst, 4096, 3, 0, 1, None, C.byref(ms)) == L.TCM_E_ARG
    assert "aligned" in lib.tcm_last_error(None).decode()
    # dst inside the three sources
    assert lib.tcm_hbm_probe(src, src + 4 * 4096, 4096, 3, 0, 1, None, C.byref(ms)) == L.TCM_E_ARG
    assert "overlaps" in lib.tcm_last_error(None).decode()
