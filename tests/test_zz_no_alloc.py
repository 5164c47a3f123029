"""tcm_read_noalloc (the read entry point that allocates nothing) against
tcm_read_shot, through the C-ABI: two reads in a row, the second of a smaller
box, both equal to the allocating read bit for bit; a box beyond the static
staging array is refused."""
import ctypes as C

import numpy as np
import pytest

import tcm_inputs as ti

pytestmark = pytest.mark.gpu
tcm = pytest.importorskip("paper_1702_00216_amd")
from paper_1702_00216_amd import _lib as L  # noqa: E402


def announce(msg):
    print(f"\n[case] {msg}", flush=True)


def _read_alloc(sim, shot, which, o, s):
    out = np.empty((s[2], s[1], s[0]), np.float32)
    rc = L.lib().tcm_read_shot(sim._h, shot, which, *o, *s, out.ctypes.data, 0)
    assert rc == 0, L.lib().tcm_last_error(sim._h)
    return out


def _read_noalloc(sim, shot, which, o, s):
    out = np.full((s[2], s[1], s[0]), np.nan, np.float32)
    rc = L.lib().tcm_read_noalloc(sim._h, shot, which, *o, *s, out.ctypes.data)
    assert rc == 0, L.lib().tcm_last_error(sim._h)
    return out


@pytest.mark.parametrize("engine", ["blocks", "dense"])
def test_noalloc_read_equals_allocating_read(engine):
    announce(f"tcm_read_noalloc vs tcm_read_shot ({engine})")
    shape = (150, 131, 97)
    c = ti.random_media(shape, seed=31, cmin=0.5, cmax=1.0)
    sim = tcm.Simulation(shape, 1.0, 0.5, c, engine=engine)
    sim.add_source((70, 60, 50), ti.ricker(0.1, 0.5).w32)
    sim.step(90)
    boxes = [((0, 0, 0), shape), ((3, 17, 40), (101, 64, 33))]      # second call: smaller box
    for which in (0, 1):
        for o, s in boxes:
            a = _read_alloc(sim, 0, which, o, s)
            b = _read_noalloc(sim, 0, which, o, s)
            assert np.array_equal(a, b) and np.abs(a).max() > 0, (which, o, s)
    sim.step(3)
    for o, s in reversed(boxes):
        assert np.array_equal(_read_alloc(sim, 0, 0, o, s), _read_noalloc(sim, 0, 0, o, s))
    sim.close()


def test_noalloc_read_of_a_batch_shot_and_limits():
    announce("tcm_read_noalloc batch shot and limits")
    shapes = [(40, 33, 20), (64, 70, 58)]
    media = [ti.random_media(s, seed=5 + i, cmin=0.5, cmax=1.0) for i, s in enumerate(shapes)]
    sim = tcm.Simulation(shapes, 1.0, 0.5, media)
    for i, s in enumerate(shapes):
        sim.add_source(tuple(v // 2 for v in s), ti.ricker(0.12, 0.5).w32, shot=i)
    sim.step(40)
    for i, s in enumerate(shapes):
        assert np.array_equal(_read_alloc(sim, i, 0, (0, 0, 0), s), _read_noalloc(sim, i, 0, (0, 0, 0), s))
    out = np.empty(4, np.float32)
    lib = L.lib()
    assert lib.tcm_read_noalloc(sim._h, 1, 0, 60, 0, 0, 5, 1, 1, out.ctypes.data) == L.TCM_E_RANGE
    assert lib.tcm_read_noalloc(sim._h, 2, 0, 0, 0, 0, 1, 1, 1, out.ctypes.data) == L.TCM_E_RANGE
    assert lib.tcm_read_noalloc(sim._h, 0, 2, 0, 0, 0, 1, 1, 1, out.ctypes.data) == L.TCM_E_ARG
    assert lib.tcm_read_noalloc(sim._h, 0, 0, 0, 0, 0, 1, 1, 1, None) == L.TCM_E_ARG
    sim.close()
    # a box of more than 8 Mi nodes is refused before any work
    big = (256, 256, 129)
    sim = tcm.Simulation(big, 1.0, 0.5, np.ones(big[::-1], np.float32))
    rc = lib.tcm_read_noalloc(sim._h, 0, 0, 0, 0, 0, *big, C.c_void_p(1))
    assert rc == L.TCM_E_ARG and b"staging" in lib.tcm_last_error(sim._h)
    small = _read_noalloc(sim, 0, 0, (0, 0, 0), (256, 256, 128))          # exactly 8 Mi nodes
    assert not small.any()
    sim.close()
