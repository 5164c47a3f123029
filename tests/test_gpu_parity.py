"""Parity of the HIP path (through the C-ABI) with the CPU oracle.

FP32 values must be bit-exact (as IEEE values, -0 == +0) to the oracle at
the same thresholds: O1 (dense) at trigger = retire = 0, O2 (CPU TCM) at any
thresholds; activation decisions are comparisons of identical values, so the
active sets and their statistics must match exactly as well.
"""
import numpy as np
import pytest

import oracle
import tcm_inputs as ti
from conftest import values_equal

pytestmark = pytest.mark.gpu
tcm = pytest.importorskip("paper_1702_00216_amd")


def announce(msg):
    print(f"\n[case] {msg}", flush=True)


def gpu_run(shape, dt, media, sources, steps, trigger=0.0, retire=0.0, receivers=None,
            engine="blocks", **kw):
    sim = tcm.Simulation(shape, 1.0, dt, media, trigger, retire, engine=engine, **kw)
    for xyz, w in sources:
        sim.add_source(xyz, w)
    if receivers is not None:
        sim.set_receivers(receivers)
    if steps:
        sim.step(steps)
    return sim


def relerr(a, b):
    return float(np.linalg.norm(a.astype(np.float64) - b) / np.linalg.norm(b))


def test_c1_bitexact_to_dense_oracle_and_fp64_error():
    announce("C1 64^3 tau=0 100 steps")
    w = ti.c1()
    src = [(w.source, w.wavelet.w32)]
    rec = [(40, 32, 32), (32, 32, 60), (5, 7, 9)]
    phi, prev, tr = oracle.dense_run(w.c_dense, w.dt, 1.0, w.steps, np.float32, sources=src,
                                     receivers=rec)
    sim = gpu_run(w.shape, w.dt, w.c_dense, src, w.steps, receivers=rec)
    assert values_equal(sim.read(0), phi)
    assert values_equal(sim.read(1), prev)
    assert values_equal(sim.read_traces(), tr)
    st = sim.stats()
    assert st["step"] == 100 and st["error"] == 0 and st["active_blocks"] == 512
    ref, _, _ = oracle.dense_run(w.c_dense, w.dt, 1.0, w.steps, np.float64,
                                 sources=[(w.source, w.wavelet.w32.astype(np.float64))])
    e = relerr(sim.read(0), ref)
    print(f"C1 rel-L2 vs FP64 = {e:.3e}")
    assert e <= 1e-5
    # work accounting matches the CPU TCM
    t = oracle.TCM(w.c_dense, w.dt, 1.0, 0.0, 0.0)
    t.add_source(w.source, w.wavelet.w32)
    t.step(w.steps)
    o = t.stats()
    assert st["cell_updates"] == o["updates"] and st["activations"] == o["activations"]
    assert st["peak_active_blocks"] == o["peak_active"]


def test_dense_engine_bitexact():
    announce("dense engine C1 + ragged heterogeneous")
    w = ti.c1()
    src = [(w.source, w.wavelet.w32)]
    phi, prev, _ = oracle.dense_run(w.c_dense, w.dt, 1.0, w.steps, np.float32, sources=src)
    sim = gpu_run(w.shape, w.dt, w.c_dense, src, w.steps, engine="dense")
    assert values_equal(sim.read(0), phi) and values_equal(sim.read(1), prev)
    shape = (70, 45, 33)
    c = ti.random_media(shape, seed=3, cmin=0.2, cmax=1.0)
    src = [((0, 44, 17), ti.ricker(0.1, 0.55).w32), ((35, 20, 32), ti.ricker(0.2, 0.55).w32)]
    phi, prev, tr = oracle.dense_run(c, 0.55, 1.0, 77, np.float32, sources=src, receivers=[(1, 2, 3)])
    sim = gpu_run(shape, 0.55, c, src, 77, engine="dense", receivers=[(1, 2, 3)])
    assert values_equal(sim.read(0), phi) and values_equal(sim.read(1), prev)
    assert values_equal(sim.read_traces(), tr)


@pytest.mark.parametrize("shape", [(37, 29, 21), (8, 8, 8), (9, 17, 65), (1, 1, 1), (130, 3, 12)])
def test_ragged_heterogeneous_tau0(shape):
    announce(f"ragged tau=0 {shape}")
    c = ti.random_media(shape, seed=sum(shape), cmin=0.3, cmax=1.0)
    dt = 0.55
    nx, ny, nz = shape
    src = [((nx // 2, ny // 2, nz // 2), ti.ricker(0.12, dt).w32),
           ((nx - 1, 0, nz - 1), -0.5 * ti.ricker(0.2, dt).w32)]
    phi, prev, _ = oracle.dense_run(c, dt, 1.0, 90, np.float32, sources=src)
    sim = gpu_run(shape, dt, c, src, 0)
    for k in range(3):          # several calls: graph and direct paths mix
        sim.step(30)
    assert values_equal(sim.read(0), phi)
    assert values_equal(sim.read(1), prev)


@pytest.mark.parametrize("trig,ret,steps", [(3e-4, 5e-5, 150), (1e-3, 1e-3, 120), (3e-3, 1e-3, 140)])
def test_thresholds_match_cpu_tcm(trig, ret, steps):
    announce(f"tau>0 vs CPU TCM trig={trig} ret={ret}")
    shape = (72, 64, 56)
    c = ti.random_media(shape, seed=9, cmin=0.8, cmax=1.0)
    w = ti.ricker(0.12, 0.5).w32
    trig, ret = np.float32(trig), np.float32(ret)
    t = oracle.TCM(c, 0.5, 1.0, trig, ret)
    t.add_source((36, 32, 28), w)
    sim = gpu_run(shape, 0.5, c, [((36, 32, 28), w)], 0, trig, ret)
    for k in range(steps // 10):
        assert t.step(10) == 0
        sim.step(10)
        o, g = t.stats(), sim.stats()
        assert g["active_blocks"] == o["active"], k
        assert g["activations"] == o["activations"] and g["retirements"] == o["retirements"]
        assert g["cell_updates"] == o["updates"]
    assert values_equal(sim.read(0), t.read(0))
    assert values_equal(sim.read(1), t.read(1))


def test_retirement_path_matches_cpu_tcm():
    """Source cell isolated by a huge threshold: it runs alone, then retires."""
    announce("isolated source block then retire")
    shape = (32, 32, 32)
    c = np.ones(shape, np.float32)
    w = ti.ricker(0.15, 0.5).w32
    big = np.float32(1e30)
    sim = gpu_run(shape, 0.5, c, [((13, 10, 9), w)], w.size - 1, big, big)
    alone, _, _ = oracle.dense_run(np.ones((8, 8, 8), np.float32), 0.5, 1.0, w.size - 1,
                                   np.float32, sources=[((5, 2, 1), w)])
    out = sim.read(0)
    assert values_equal(out[8:16, 8:16, 8:16], alone)
    out[8:16, 8:16, 8:16] = 0
    assert not out.any()
    sim.step(1)
    st = sim.stats()
    assert st["active_blocks"] == 0 and st["retirements"] == 1
    assert not sim.read(0).any()


@pytest.mark.parametrize("levels,w", [((0.0, 0.0), (0.25, -0.5)), ((1e30, 0.125), (0.25, -0.5)),
                                      ((0.25, 0.0), (0.25, -0.25)),
                                      ((float(np.nextafter(np.float32(0.25), np.float32(0))), 0.0),
                                       (0.25, -0.25)),
                                      ((1e30, 0.25), (0.25, -0.25)),
                                      ((1e30, float(np.nextafter(np.float32(0.25), np.float32(0)))),
                                       (0.25, -0.25))])
def test_exact_level_cases_match_cpu_tcm(levels, w):
    """C2 = 0, so the field changes only at its source node: a value exactly at
    the trigger or keep level (strict comparisons), one ulp above it, and a
    cell whose new level is zero while its current level is not (kept at
    threshold 0).  Active sets and fields equal the CPU TCM every step."""
    announce(f"exact-level rules {levels} w={w}")
    trig, ret = (np.float32(v) for v in levels)
    c = np.zeros((24, 16, 16), np.float32)
    ws = np.array(w, np.float32)
    xyz = (7, 3, 3) if ws[1] == -ws[0] else (3, 4, 5)
    t = oracle.TCM(c, 0.5, 1.0, trig, ret)
    t.add_source(xyz, ws)
    sim = gpu_run((16, 16, 24), 0.5, c, [(xyz, ws)], 0, trig, ret)
    for k in range(8):
        assert t.step(1) == 0
        sim.step(1)
        assert sim.stats()["active_blocks"] == t.stats()["active"], k
        assert values_equal(sim.read(0), t.read(0)) and values_equal(sim.read(1), t.read(1)), k
    g, o = sim.stats(), t.stats()
    assert g["activations"] == o["activations"] and g["retirements"] == o["retirements"]


def test_retiring_pulse_matches_cpu_tcm_every_step():
    """Homogeneous box at a single level: the pulse leaves cells behind it,
    some released one step after their new level fell below the level."""
    announce("retiring pulse, single level, every step")
    shape = (56, 52, 48)
    c = np.ones(shape[::-1], np.float32)
    w = ti.ricker(0.15, 0.5).w32
    lvl = np.float32(3e-3 * float(np.max(np.abs(w))))
    t = oracle.TCM(c, 0.5, 1.0, lvl, lvl)
    t.add_source((20, 18, 15), w)
    sim = gpu_run(shape, 0.5, c, [((20, 18, 15), w)], 0, lvl, lvl)
    for k in range(90):
        assert t.step(1) == 0
        sim.step(1)
        assert sim.stats()["active_blocks"] == t.stats()["active"], k
    assert values_equal(sim.read(0), t.read(0)) and values_equal(sim.read(1), t.read(1))
    g, o = sim.stats(), t.stats()
    assert o["retirements"] > 0 and g["retirements"] == o["retirements"]
    assert g["cell_updates"] == o["updates"]


@pytest.mark.parametrize("path,interval", [("two-launch", 1), ("three-pass", 1), ("three-pass", 8)])
def test_source_pin_keeps_quiet_blocks(path, interval):
    """A source whose wavelet starts with 24 zero samples: its block is kept
    by its pin while the field there is below every level (and, with the
    update every 8 steps, counts as hot, so its 26 neighbours are kept too),
    then the pulse runs.  Active sets every step, counters and fields equal
    the CPU TCM on both update paths."""
    announce(f"source pin on a quiet block, {path}, interval {interval}")
    shape = (48, 40, 40)
    c = np.ones(shape[::-1], np.float32)
    w = np.concatenate([np.zeros(24, np.float32), ti.ricker(0.15, 0.5).w32])
    lvl = np.float32(3e-3 * float(np.max(np.abs(w))))
    xyz = (20, 18, 15)
    t = oracle.TCM(c, 0.5, 1.0, lvl, lvl, interval=interval)
    t.add_source(xyz, w)
    sim = gpu_run(shape, 0.5, c, [(xyz, w)], 0, lvl, lvl, trigger_interval=interval,
                  three_pass_update=path == "three-pass")
    for k in range(40):
        assert t.step(1) == 0
        sim.step(1)
        assert sim.stats()["active_blocks"] == t.stats()["active"], k
    assert t.step(80) == 0          # the pulse fills the box; some blocks retire
    sim.step(80)
    g, o = sim.stats(), t.stats()
    assert g["active_blocks"] == o["active"]
    assert g["activations"] == o["activations"] and g["retirements"] == o["retirements"]
    assert g["cell_updates"] == o["updates"]
    assert values_equal(sim.read(0), t.read(0)) and values_equal(sim.read(1), t.read(1))
    sim.close()


def test_pool_cap_fails_like_cpu_tcm():
    announce("pool cap E_POOL")
    w = ti.c1(steps=60)
    cap = 100
    t = oracle.TCM(w.c_dense, w.dt, 1.0, 0.0, 0.0, cap=cap)
    t.add_source(w.source, w.wavelet.w32)
    assert t.step(60) == oracle.TCM.E_POOL
    o = t.stats()
    sim = gpu_run(w.shape, w.dt, w.c_dense, [(w.source, w.wavelet.w32)], 0, pool_bytes=cap * 6144)
    with pytest.raises(tcm.TCMError) as ei:
        sim.step(60)
    assert ei.value.status == -3
    g = sim.stats()
    assert g["step"] == o["step"] and g["active_blocks"] == o["active"] and g["error"] == -3
    assert values_equal(sim.read(0), t.read(0))
    assert values_equal(sim.read(1), t.read(1))
    assert sim.step_status(3) == -3 and sim.stats()["step"] == o["step"]


@pytest.mark.parametrize("slack", [0, -1])
def test_pool_exact_fit_hands_released_slots_over(slack):
    """A pool of exactly the peak active count: at step 45 the step's new
    blocks exceed the free slots and released slots are handed over directly
    (placement wraps the key range over 47 slots).  One slot fewer fails with
    E_POOL at the same step as the CPU TCM with that cap."""
    announce(f"pool of peak{slack:+d} slots, released slots handed over")
    shape = (48, 32, 32)
    c = np.ones(shape[::-1], np.float32)
    w = ti.ricker(0.15, 0.5).w32
    lev = np.float32(3e-2)
    ref = oracle.TCM(c, 0.5, 1.0, lev, lev)
    ref.add_source((10, 16, 16), w)
    assert ref.step(200) == 0
    cap = ref.stats()["peak_active"] + slack
    t = oracle.TCM(c, 0.5, 1.0, lev, lev, cap=cap)
    t.add_source((10, 16, 16), w)
    rc = t.step(200)
    assert rc == (0 if slack == 0 else oracle.TCM.E_POOL)
    sim = gpu_run(shape, 0.5, c, [((10, 16, 16), w)], 0, lev, lev, pool_bytes=cap * 6144)
    assert sim.step_status(200) == rc
    g, o = sim.stats(), t.stats()
    assert g["step"] == o["step"] and g["active_blocks"] == o["active"]
    assert g["activations"] == o["activations"] and g["retirements"] == o["retirements"]
    assert g["cell_updates"] == o["updates"]
    assert values_equal(sim.read(0), t.read(0)) and values_equal(sim.read(1), t.read(1))


def test_zero_speed_region_and_no_source():
    """c = 0 inside a box (C2 = 0 there: phi^{n+1} = 2 phi^n - phi^{n-1}),
    at threshold 0 (dense oracle) and above it (CPU TCM); a handle without a
    source stays empty."""
    announce("zero-speed box; no source")
    shape = (40, 36, 44)
    c = ti.random_media(shape, seed=12, cmin=0.4, cmax=1.0)
    c[10:26, 8:30, 20:33] = 0.0
    w = ti.ricker(0.12, 0.5).w32
    src = [((12, 18, 16), w)]
    phi, prev, _ = oracle.dense_run(c, 0.5, 1.0, 90, np.float32, sources=src)
    sim = gpu_run(shape, 0.5, c, src, 90)
    assert values_equal(sim.read(0), phi) and values_equal(sim.read(1), prev)
    lev = np.float32(1e-3)
    t = oracle.TCM(c, 0.5, 1.0, lev, np.float32(2e-4))
    t.add_source(*src[0])
    assert t.step(90) == 0
    sim = gpu_run(shape, 0.5, c, src, 90, lev, np.float32(2e-4))
    assert values_equal(sim.read(0), t.read(0))
    assert sim.stats()["cell_updates"] == t.stats()["updates"]
    empty = gpu_run(shape, 0.5, c, [], 0)
    assert not empty.read(0).any()
    empty.step(25)
    st = empty.stats()
    assert st["step"] == 25 and st["active_blocks"] == 0 and st["cell_updates"] == 0
    assert not empty.read(0).any() and not empty.read(1).any()


def test_layered_and_lattice_media():
    announce("layered + lattice media")
    shape = (48, 40, 64)
    lay = ti.LayeredMedia(np.array([0, 20, 41], np.int32), np.array([1500, 3000, 2200], np.float32))
    dt = 0.5 / 3000
    wv = ti.ricker(300.0, dt).w32
    src = [((24, 20, 18), wv)]
    phi, prev, _ = oracle.dense_run(lay.dense(*shape), dt, 1.0, 120, np.float32, sources=src)
    sim = gpu_run(shape, dt, lay, src, 120)
    assert values_equal(sim.read(0), phi) and values_equal(sim.read(1), prev)
    lat = ti.lognormal_lattice(shape, seed=12, sigma=6.0, spacing=4)
    dt = 0.5 / 4500
    cd = ti.lattice_to_dense(lat, shape)
    wv = ti.ricker(250.0, dt).w32
    src = [((10, 30, 50), wv)]
    phi, prev, _ = oracle.dense_run(cd, dt, 1.0, 130, np.float32, sources=src)
    sim = gpu_run(shape, dt, lat, src, 130)
    assert values_equal(sim.read(0), phi) and values_equal(sim.read(1), prev)
    dsim = gpu_run(shape, dt, lat, src, 130, engine="dense")
    assert values_equal(dsim.read(0), phi)


def test_subnormal_values_are_kept():
    """Tiny source amplitudes drive the field into FP32 subnormals; flushing
    them to zero on either side would break equality."""
    announce("subnormals")
    shape = (24, 24, 24)
    c = np.ones(shape, np.float32)
    w = (ti.ricker(0.15, 0.5).w64 * 1e-39).astype(np.float32)
    assert np.any((np.abs(w) < np.finfo(np.float32).tiny) & (w != 0))
    phi, _, _ = oracle.dense_run(c, 0.5, 1.0, 60, np.float32, sources=[((12, 12, 12), w)])
    assert np.any((np.abs(phi) < np.finfo(np.float32).tiny) & (phi != 0))
    sim = gpu_run(shape, 0.5, c, [((12, 12, 12), w)], 60)
    assert values_equal(sim.read(0), phi)
    dsim = gpu_run(shape, 0.5, c, [((12, 12, 12), w)], 60, engine="dense")
    assert values_equal(dsim.read(0), phi)


def test_launch_modes_and_reads_agree():
    announce("graphs / no graphs / timing / step splits / box + device reads")
    import torch
    w = ti.c1(steps=64)
    src = [(w.source, w.wavelet.w32)]
    phi, _, _ = oracle.dense_run(w.c_dense, w.dt, 1.0, 64, np.float32, sources=src)
    a = gpu_run(w.shape, w.dt, w.c_dense, src, 64, graph_steps=8)
    b = gpu_run(w.shape, w.dt, w.c_dense, src, 0, graphs=False)
    for k in range(64):
        b.step(1)
    c = gpu_run(w.shape, w.dt, w.c_dense, src, 64, timing=True)
    # timed runs split over calls, without graphs, and with the update every
    # 4 steps from a step that is not on the interval boundary
    d = gpu_run(w.shape, w.dt, w.c_dense, src, 0, timing=True, graph_steps=24)
    d.step(5)
    d.step(59)
    e = gpu_run(w.shape, w.dt, w.c_dense, src, 64, timing=True, graphs=False)
    f = gpu_run(w.shape, w.dt, w.c_dense, src, 0, timing=True, trigger_interval=4, graph_steps=8)
    f.step(3)
    f.step(61)
    for s in (a, b, c, d, e, f):
        assert values_equal(s.read(0), phi)
    for s in (c, d, e, f):
        assert s.stats()["stencil_launches"] == 64 and s.stats()["stencil_ms"] > 0
        assert s.stats()["stencil_cells"] == s.stats()["cell_updates"]
    for s in (d, e, f):
        s.close()
    box = a.read(0, box=((3, 17, 30), (20, 9, 11)))
    assert values_equal(box, phi[30:41, 17:26, 3:23])
    out = torch.empty(11 * 9 * 20, dtype=torch.float32, device="cuda")
    a.read(0, box=((3, 17, 30), (20, 9, 11)), out=out)
    assert values_equal(out.cpu().numpy().reshape(11, 9, 20), phi[30:41, 17:26, 3:23])
    # even x origin and width: two nodes per thread; odd width, or an output
    # that is not 8-byte aligned: one node per thread
    assert values_equal(a.read(0, box=((4, 17, 30), (20, 9, 11))), phi[30:41, 17:26, 4:24])
    assert values_equal(a.read(0, box=((4, 17, 30), (19, 9, 11))), phi[30:41, 17:26, 4:23])
    big = torch.empty(1 + 11 * 9 * 20, dtype=torch.float32, device="cuda")
    a.read(0, box=((4, 17, 30), (20, 9, 11)), out=big[1:])
    assert values_equal(big[1:].cpu().numpy().reshape(11, 9, 20), phi[30:41, 17:26, 4:24])
    assert values_equal(a.read(1, box=((56, 0, 60), (8, 64, 4))), a.read(1)[60:64, :, 56:64])
    a.reset()
    assert not a.read(0).any() and a.stats()["step"] == 0
    a.add_source(w.source, w.wavelet.w32)
    a.step(64)
    assert values_equal(a.read(0), phi)


@pytest.mark.parametrize("tile,per_wave", [(2, 1), (4, 1), (8, 1), (4, 2), (8, 2)])
def test_workgroup_tiles_agree_with_oracle(tile, per_wave):
    """Every stencil workgroup tile (2, 4 or 8 x-adjacent blocks sharing x
    faces through LDS; one or two blocks per wave), with a few workgroups per
    CU so that waves of one workgroup meet ragged list ends, equals the CPU
    TCM at a threshold and the dense oracle at threshold 0 (random media,
    ragged grid)."""
    announce(f"workgroup tile {tile}, {per_wave} per wave")
    shape = (45, 38, 27)
    c = ti.random_media(shape, seed=31, cmin=0.3, cmax=1.0)
    src = [((20, 17, 11), ti.ricker(0.12, 0.5).w32), ((44, 0, 26), ti.ricker(0.2, 0.5).w32)]
    phi, prev, _ = oracle.dense_run(c, 0.5, 1.0, 110, np.float32, sources=src)
    for wpc in (1, 3):
        sim = gpu_run(shape, 0.5, c, src, 110, blocks_per_wg=tile, blocks_per_wave=per_wave, wg_per_cu=wpc)
        assert values_equal(sim.read(0), phi) and values_equal(sim.read(1), prev)
    lev = np.float32(3e-4)
    t = oracle.TCM(c, 0.5, 1.0, lev, np.float32(5e-5))
    for xyz, w in src:
        t.add_source(xyz, w)
    assert t.step(110) == 0
    sim = gpu_run(shape, 0.5, c, src, 110, lev, np.float32(5e-5), blocks_per_wg=tile,
                  blocks_per_wave=per_wave, timing=True)
    assert values_equal(sim.read(0), t.read(0))
    g, o = sim.stats(), t.stats()
    assert g["cell_updates"] == o["updates"] and g["activations"] == o["activations"]


def test_caller_pool_and_stream():
    """The pool in a caller's torch tensor and the work on a caller's torch
    stream (steps, reads into a CUDA tensor); two handles on separate streams
    stay independent."""
    announce("caller device pool + torch streams")
    import torch
    w = ti.c1(steps=70)
    src = [(w.source, w.wavelet.w32)]
    phi, _, _ = oracle.dense_run(w.c_dense, w.dt, 1.0, 70, np.float32, sources=src)
    slots = 512
    pool = torch.empty(slots * 1536, dtype=torch.float32, device="cuda")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    a = gpu_run(w.shape, w.dt, w.c_dense, src, 0, device_pool=pool, pool_bytes=slots * 6144, stream=s1)
    b = gpu_run(w.shape, w.dt, w.c_dense, src, 0, stream=s2)
    for k in range(7):
        a.step(10)
        b.step(10)
    out = torch.empty(w.shape[0] * w.shape[1] * w.shape[2], dtype=torch.float32, device="cuda")
    with torch.cuda.stream(s1):
        a.read(0, out=out)
    torch.cuda.synchronize()
    assert values_equal(out.cpu().numpy().reshape(phi.shape), phi)
    assert values_equal(b.read(0), phi)
    assert a.stats()["pool_bytes"] == slots * 6144


@pytest.mark.parametrize("engine,interval", [("blocks", 1), ("blocks", 8), ("dense", 1)])
def test_snapshot_restore_repeats_the_run(engine, interval):
    """Snapshot at step 37, step on, restore, step again: the same fields,
    statistics and traces; a snapshot of another handle and a restore after
    a new source are refused."""
    announce(f"snapshot / restore ({engine}, interval {interval})")
    w = ti.c1(steps=100)
    src = [(w.source, w.wavelet.w32)]
    lev = np.float32(1e-4 if engine == "blocks" else 0.0)
    sim = gpu_run(w.shape, w.dt, w.c_dense, src, 0, lev, np.float32(lev / 5), engine=engine,
                  receivers=[(3, 4, 5), (32, 40, 10)], trigger_interval=interval)
    sim.step(37)
    snap = sim.snapshot()
    sim.step(45)
    first = (sim.read(0), sim.read(1), sim.stats(), sim.read_traces())
    sim.restore(snap)
    assert sim.stats()["step"] == 37
    sim.step(20)
    sim.step(25)
    again = (sim.read(0), sim.read(1), sim.stats(), sim.read_traces())
    assert values_equal(first[0], again[0]) and values_equal(first[1], again[1])
    for k in ("step", "active_blocks", "cell_updates", "activations", "retirements"):
        assert first[2][k] == again[2][k], k
    assert values_equal(first[3], again[3])
    other = gpu_run(w.shape, w.dt, w.c_dense, src, 0, engine=engine)
    with pytest.raises(tcm.TCMError) as ei:
        other.restore(snap)
    assert ei.value.status == -1
    sim.add_source((10, 10, 10), w.wavelet.w32)
    with pytest.raises(tcm.TCMError) as ei:
        sim.restore(snap)
    assert ei.value.status == -6
    snap.close()


def test_source_added_mid_run():
    announce("source added after 30 steps")
    w = ti.c1(steps=80)
    w2 = ti.ricker(0.2, w.dt).w32
    # oracle: second source starts at step 30
    phi, prev, _ = oracle.dense_run(w.c_dense, w.dt, 1.0, 80, np.float32,
                                    sources=[(w.source, w.wavelet.w32), ((10, 50, 20), w2, 30)])
    sim = gpu_run(w.shape, w.dt, w.c_dense, [(w.source, w.wavelet.w32)], 30)
    sim.add_source((10, 50, 20), w2)
    sim.step(50)
    assert values_equal(sim.read(0), phi) and values_equal(sim.read(1), prev)


def test_input_errors_are_reported():
    announce("error paths")
    c = np.ones((16, 16, 16), np.float32)
    sim = tcm.Simulation((16, 16, 16), 1.0, 0.5, c)
    with pytest.raises(tcm.TCMError) as ei:
        sim.add_source((16, 0, 0), np.ones(3, np.float32))
    assert ei.value.status == -4
    with pytest.raises(tcm.TCMError) as ei:
        sim.set_receivers([(0, 0, -1)])
    assert ei.value.status == -4
    with pytest.raises(tcm.TCMError) as ei:
        sim.read(0, box=((10, 0, 0), (7, 1, 1)))
    assert ei.value.status == -4
    with pytest.raises(tcm.TCMError) as ei:
        tcm.Simulation((16, 16, 16), 1.0, 0.6, c)
    assert ei.value.status == -2


def test_uniform_c2_blocks_give_identical_results():
    """Blocks whose C2 is uniform read it as one scalar (the paper's hybrid
    engine for homogeneous cells); values are identical either way."""
    announce("uniform-C2 blocks on/off")
    shape = (70, 45, 60)                          # partial blocks in x, y and z
    lay = ti.LayeredMedia(np.array([0, 24, 37], np.int32), np.array([1500, 3000, 2200], np.float32))
    dt = 0.5 / 3000
    src = [((33, 20, 30), ti.ricker(300.0, dt).w32)]
    trig, ret = np.float32(1e-5), np.float32(1e-6)
    a = gpu_run(shape, dt, lay, src, 150, trig, ret, timing=True)
    b = gpu_run(shape, dt, lay, src, 150, trig, ret, uniform_c2=False, timing=True)
    assert values_equal(a.read(0), b.read(0)) and values_equal(a.read(1), b.read(1))
    t = oracle.TCM(lay.dense(*shape), dt, 1.0, trig, ret)
    t.add_source(*src[0])
    t.step(150)
    assert values_equal(a.read(0), t.read(0))
    sa, sb = a.stats(), b.stats()
    assert sa["cell_updates"] == sb["cell_updates"] == t.stats()["updates"]
    assert sb["uniform_cell_updates"] == 0
    # blocks straddling z = 37 (not a multiple of 8) or cut by the domain edge are not uniform
    assert 0 < sa["uniform_cell_updates"] < sa["cell_updates"]
    assert 0 < sa["stencil_cells_uniform"] <= sa["stencil_cells"]
    # the timed launches stepped exactly the nodes the run counts as updated,
    # over several calls as well
    for n in (7, 1, 30):
        a.step(n)
        sa = a.stats()
        assert sa["stencil_cells"] == sa["cell_updates"], n
        assert sa["stencil_cells_uniform"] == sa["uniform_cell_updates"], n
        assert sa["stencil_launches"] == sa["step"], n


@pytest.mark.parametrize("n,alpha", [(20, 0.8), (3, 0.0), (1, 1.0)])
def test_shutdown_decay_matches_cpu_tcm(n, alpha):
    announce(f"shutdown decay n={n} alpha={alpha}")
    shape = (72, 64, 56)
    c = ti.random_media(shape, seed=9, cmin=0.8, cmax=1.0)
    w = ti.ricker(0.12, 0.5).w32
    trig, ret = np.float32(3e-3), np.float32(1e-3)
    t = oracle.TCM(c, 0.5, 1.0, trig, ret, shutdown_steps=n, shutdown_alpha=np.float32(alpha))
    t.add_source((36, 32, 28), w)
    sim = gpu_run(shape, 0.5, c, [((36, 32, 28), w)], 0, trig, ret, shutdown_steps=n,
                  shutdown_alpha=alpha)
    for k in range(14):
        assert t.step(10) == 0
        sim.step(10)
        o, g = t.stats(), sim.stats()
        assert g["active_blocks"] == o["active"], k
        assert g["activations"] == o["activations"] and g["retirements"] == o["retirements"], k
        assert g["cell_updates"] == o["updates"], k
    assert values_equal(sim.read(0), t.read(0))
    assert values_equal(sim.read(1), t.read(1))


def test_shutdown_total_attenuation_eq6_on_gpu():
    announce("eq.(6) A = alpha^n on the GPU")
    c = np.ones((16, 16, 16), np.float32)
    sim = gpu_run((16, 16, 16), 0.0, c, [((3, 3, 3), np.array([1.0, -1.0], np.float32))], 0,
                  2.0, 2.0, shutdown_steps=5, shutdown_alpha=0.5)
    vals = []
    for k in range(8):
        sim.step(1)
        vals.append(float(sim.read(0)[3, 3, 3]))
    assert vals[:7] == [1.0, 0.5, 0.25, 0.125, 0.0625, 0.03125, 0.0]
    st = sim.stats()
    assert st["active_blocks"] == 0 and st["decay_block_steps"] == 5


@pytest.mark.parametrize("rt,rr,n", [(1e-3, 1e-4, 0), (3e-2, 3e-2, 0), (1e-3, 2e-4, 10)])
def test_adaptive_levels_match_cpu_tcm(rt, rr, n):
    """Levels relative to the domain maximum (Table 1 Trig_level): the GPU uses
    the same per-step levels and makes the same decisions as the CPU TCM."""
    announce(f"adaptive levels rel {rt}/{rr} shutdown {n}")
    shape = (72, 64, 56)
    c = ti.random_media(shape, seed=9, cmin=0.8, cmax=1.0)
    w = ti.ricker(0.12, 0.5).w32
    rt, rr = np.float32(rt), np.float32(rr)
    t = oracle.TCM(c, 0.5, 1.0, 0.0, 0.0, trigger_rel=rt, retire_rel=rr, shutdown_steps=n,
                   shutdown_alpha=np.float32(0.7))
    t.add_source((36, 32, 28), w)
    sim = gpu_run(shape, 0.5, c, [((36, 32, 28), w)], 0, trigger_rel=rt, retire_rel=rr,
                  shutdown_steps=n, shutdown_alpha=0.7)
    for k in range(30):
        assert t.step(5) == 0
        sim.step(5)
        o, g = t.stats(), sim.stats()
        assert (g["trigger_level"], g["retire_level"]) == t.levels(), k
        assert g["active_blocks"] == o["active"], k
        assert g["activations"] == o["activations"] and g["retirements"] == o["retirements"], k
        assert g["cell_updates"] == o["updates"], k
    assert values_equal(sim.read(0), t.read(0))
    assert values_equal(sim.read(1), t.read(1))


@pytest.mark.parametrize("k", [2, 5, 8])
def test_update_interval_exact_at_tau0(k):
    """Activation update every k steps with the 26-block lookahead: threshold
    0 stays equal to the dense grid, through graph replays and direct steps."""
    announce(f"update interval {k} at tau=0")
    shape = (37, 29, 21)
    c = ti.random_media(shape, seed=7, cmin=0.3, cmax=1.0)
    dt = 0.55
    srcs = [((16, 8, 8), ti.ricker(0.12, dt).w32), ((36, 0, 20), -0.5 * ti.ricker(0.2, dt).w32)]
    phi, prev, tr = oracle.dense_run(c, dt, 1.0, 97, np.float32, sources=srcs, receivers=[(3, 4, 5)])
    sim = gpu_run(shape, dt, c, srcs, 0, trigger_interval=k, graph_steps=8, receivers=[(3, 4, 5)])
    for chunk in (13, 40, 44):
        sim.step(chunk)
    assert values_equal(sim.read(0), phi) and values_equal(sim.read(1), prev)
    assert values_equal(sim.read_traces(), tr)


@pytest.mark.parametrize("k", [4, 8])
def test_self_advancing_steps_equal_advance_launches(k):
    """Steps without an activation update: with no receivers the stencil's
    last workgroup advances the step, with receivers a k_advance launch does
    (and records them); fields, active sets and counters are the same."""
    announce(f"self-advancing steps vs k_advance, interval {k}")
    w = ti.c1(steps=64)
    src = [(w.source, w.wavelet.w32)]
    lvl = np.float32(3e-3 * float(np.max(np.abs(w.wavelet.w32))))
    a = gpu_run(w.shape, w.dt, w.c_dense, src, 0, lvl, lvl / 3, trigger_interval=k)
    b = gpu_run(w.shape, w.dt, w.c_dense, src, 0, lvl, lvl / 3, trigger_interval=k,
                receivers=np.array([[w.source[0] + 5, w.source[1], w.source[2]]], np.int32))
    for n in (5, 27, 40):
        a.step(n)
        b.step(n)
        sa, sb = a.stats(), b.stats()
        for key in ("step", "active_blocks", "cell_updates", "activations", "retirements"):
            assert sa[key] == sb[key], (n, key)
        assert values_equal(a.read(0), b.read(0)) and values_equal(a.read(1), b.read(1)), n
    assert np.any(b.read_traces() != 0)
    a.close()
    b.close()


@pytest.mark.parametrize("k,rel,n", [(8, False, 0), (4, True, 0), (8, False, 5)])
def test_update_interval_matches_cpu_tcm(k, rel, n):
    announce(f"update interval {k} vs CPU TCM (adaptive {rel}, shutdown {n})")
    shape = (72, 64, 56)
    c = ti.random_media(shape, seed=9, cmin=0.8, cmax=1.0)
    w = ti.ricker(0.12, 0.5).w32
    kw = dict(trigger_rel=np.float32(1e-3), retire_rel=np.float32(1e-4)) if rel else {}
    trig, ret = (0.0, 0.0) if rel else (np.float32(3e-3), np.float32(1e-3))
    t = oracle.TCM(c, 0.5, 1.0, trig, ret, interval=k, shutdown_steps=n,
                   shutdown_alpha=np.float32(0.6), **kw)
    t.add_source((36, 32, 28), w)
    sim = gpu_run(shape, 0.5, c, [((36, 32, 28), w)], 0, trig, ret, trigger_interval=k,
                  shutdown_steps=n, shutdown_alpha=0.6, **kw)
    for step in (3, 17, 40, 40, 40):
        assert t.step(step) == 0
        sim.step(step)
        o, g = t.stats(), sim.stats()
        assert g["active_blocks"] == o["active"]
        assert g["activations"] == o["activations"] and g["retirements"] == o["retirements"]
        assert g["cell_updates"] == o["updates"]
    assert values_equal(sim.read(0), t.read(0)) and values_equal(sim.read(1), t.read(1))


@pytest.mark.parametrize("seed", list(range(40)))
def test_random_configurations_match_cpu_tcm(seed):
    """Seeded random problems: ragged shape, random or z-layered media, two or
    three sources (one added mid-run), levels, update interval, shutdown decay,
    relative levels, uniform-C2 switch and workgroup tile.  Both field levels
    and the work statistics equal the CPU TCM."""
    rng = np.random.default_rng(1000 + seed)
    shape = tuple(int(v) for v in rng.integers(5, 60, size=3))
    if rng.random() < 0.5:
        c = ti.random_media(shape, seed=2000 + seed, cmin=float(rng.uniform(0.2, 0.6)), cmax=1.0)
    else:
        c = np.full(shape[::-1], 0.6, np.float32)
        c[int(rng.integers(0, shape[2])):] = 1.0
    dt = 0.55
    tr = float(rng.choice([0.0, 1e-4, 1e-3, 1e-2]))
    trig = np.float32(tr)
    ret = np.float32(tr * float(rng.choice([1.0, 0.3, 0.1])))
    interval = int(rng.choice([1, 1, 2, 3, 8]))
    sd = int(rng.choice([0, 0, 3, 10]))
    alpha = np.float32(rng.choice([0.5, 0.9]))
    rel = bool(rng.random() < 0.25)
    trel, rrel = (np.float32(1e-3), np.float32(2e-4)) if rel else (np.float32(0), np.float32(0))
    tile = int(rng.choice([2, 4, 8]))
    per_wave = 1 + (seed // 2) % 2 if tile > 2 else 1     # not drawn: the other choices stay as they were
    unif = bool(rng.random() < 0.7)
    srcs = [(tuple(int(rng.integers(0, e)) for e in shape), ti.ricker(float(rng.uniform(0.08, 0.2)), dt).w32)
            for _ in range(int(rng.integers(1, 3)))]
    late = (tuple(int(rng.integers(0, e)) for e in shape), ti.ricker(0.15, dt).w32)
    n1, n2 = int(rng.integers(10, 50)), int(rng.integers(10, 140))
    kw = dict(shutdown_steps=sd, shutdown_alpha=alpha, trigger_rel=trel, retire_rel=rrel, interval=interval)

    def oracle_run(cap=0):
        t = oracle.TCM(c, dt, 1.0, trig, ret, cap=cap, **kw)
        for xyz, w in srcs:
            t.add_source(xyz, w)
        assert t.step(n1) == 0
        t.add_source(*late)
        assert t.step(n2) == 0
        return t

    t = oracle_run()
    # every third problem runs in a pool of just above its peak block count
    # (at least 64 slots): tiles placed at hashed slot groups, probing, hand-offs
    cap = 0
    if seed % 3 == 0:
        cap = max(64, t.stats()["peak_active"] + int(rng.integers(0, 20)))
        t = oracle_run(cap)
    announce(f"random {seed}: shape {shape} levels {tr:g}/{float(ret):g} k {interval} shutdown {sd} "
             f"rel {rel} tile {tile}x{per_wave} uniform {unif} pool {cap or 'auto'} three-pass {seed % 4 == 1}")
    three = seed % 4 == 1      # where the two-launch update applies, also run the three-pass one
    sim = tcm.Simulation(shape, 1.0, dt, c, trig, ret, shutdown_steps=sd, shutdown_alpha=float(alpha),
                         trigger_rel=float(trel), retire_rel=float(rrel), trigger_interval=interval,
                         blocks_per_wg=tile, blocks_per_wave=per_wave, uniform_c2=unif, timing=bool(seed % 2),
                         pool_bytes=cap * 6144, three_pass_update=three, debug_checks=seed % 5 == 0)
    for xyz, w in srcs:
        sim.add_source(xyz, w)
    sim.step(n1)
    assert sim.check() == 0
    sim.add_source(*late)
    assert sim.check() == 0
    sim.step(n2)
    assert sim.check() == 0
    assert values_equal(sim.read(0), t.read(0)) and values_equal(sim.read(1), t.read(1))
    g, o = sim.stats(), t.stats()
    assert g["step"] == o["step"] and g["active_blocks"] == o["active"]
    assert g["activations"] == o["activations"] and g["retirements"] == o["retirements"]
    assert g["cell_updates"] == o["updates"]


@pytest.mark.parametrize("levels", [(0.0, 0.0), (3e-3, 3e-3), (1e-3, 1e-4)])
def test_two_launch_update_equals_three_pass_every_step(levels):
    """The two-launch activation update (one slot per key, constant levels,
    update every step) and the three-pass update give the same active counts
    and work every step and the same fields, with a batch of two shots, a
    source added mid-run, receivers, and a snapshot restored mid-run."""
    announce(f"two-launch vs three-pass update {levels}")
    shapes = [(70, 45, 60), (33, 81, 24)]
    media = [ti.random_media(s, seed=50 + i, cmin=0.5, cmax=1.0) for i, s in enumerate(shapes)]
    w = ti.ricker(0.12, 0.5).w32
    trig, ret = (np.float32(v) for v in levels)
    sims = [tcm.Simulation(shapes, 1.0, 0.5, media, trig, ret, three_pass_update=tp, debug_checks=True)
            for tp in (False, True)]
    for sim in sims:
        sim.add_source((35, 20, 30), w, shot=0)
        sim.add_source((16, 40, 12), -0.5 * w, shot=1)
        sim.set_receivers([(35, 25, 30), (3, 3, 3), (16, 60, 12)], shots=[0, 0, 1])
    for k in range(150):
        for sim in sims:
            if k == 60:
                sim.add_source((5, 5, 5), w, shot=1)
            sim.step(1)
        a, b = sims[0].stats(), sims[1].stats()
        for key in ("step", "active_blocks", "activations", "retirements", "cell_updates", "peak_active_blocks"):
            assert a[key] == b[key], (k, key)
        if k == 90:
            snaps = [sim.snapshot() for sim in sims]
    for sim, snap in zip(sims, snaps):
        ref = (sim.read(0, shot=1), sim.read_traces())
        sim.restore(snap)
        sim.step(59)
        assert values_equal(sim.read(0, shot=1), ref[0]) and values_equal(sim.read_traces(), ref[1])
    for shot in (0, 1):
        assert values_equal(sims[0].read(0, shot=shot), sims[1].read(0, shot=shot))
        assert values_equal(sims[0].read(1, shot=shot), sims[1].read(1, shot=shot))
    assert values_equal(sims[0].read_traces(), sims[1].read_traces())


def test_two_launch_update_over_many_runs_of_chunks():
    """A batch of three shots with 225 groups of 256 keys (15 runs of 16
    groups, whose sums give each compaction workgroup its offset): the
    two-launch update and the three-pass update give the same counts and work
    every step and the same fields, as the wave crosses the runs."""
    announce("two-launch vs three-pass update, 225 key groups")
    shapes = [(200, 180, 160), (150, 210, 130), (256, 256, 256)]
    media = [ti.random_media(s, seed=60 + i, cmin=0.5, cmax=1.0) for i, s in enumerate(shapes)]
    w = ti.ricker(0.1, 0.5).w32
    sims = [tcm.Simulation(shapes, 1.0, 0.5, media, np.float32(1e-4), np.float32(1e-5), three_pass_update=tp)
            for tp in (False, True)]
    for sim in sims:
        sim.add_source((100, 90, 80), w, shot=0)
        sim.add_source((75, 105, 65), -w, shot=1)
        sim.add_source((128, 130, 126), w, shot=2)
        sim.add_source((20, 240, 30), 0.5 * w, shot=2)
    keys = ("step", "active_blocks", "activations", "retirements", "cell_updates", "peak_active_blocks")
    for k in range(160):
        for sim in sims:
            sim.step(1)
        a, b = sims[0].stats(), sims[1].stats()
        for key in keys:
            assert a[key] == b[key], (k, key)
    assert sims[0].stats()["active_blocks"] > 2000
    assert sims[0].check() == 0
    for shot in range(3):
        assert values_equal(sims[0].read(0, shot=shot), sims[1].read(0, shot=shot))
        assert values_equal(sims[0].read(1, shot=shot), sims[1].read(1, shot=shot))


def test_two_launch_update_with_run_sums():
    """Five 512^3 shots in one handle: 5120 groups of 256 keys, beyond the
    4096 whose counts a compaction workgroup sums directly, so the plan also
    sums runs of 16 groups with device atomics and the compaction takes its
    offset from those.  Counts and work equal the three-pass update every
    step, and the fields equal it at the end."""
    announce("two-launch (run sums) vs three-pass update, 5 x 512^3 shots")
    shapes = [(512, 512, 512)] * 5
    lay = ti.LayeredMedia(np.array([0, 200, 330], np.int32), np.array([1500, 3000, 2200], np.float32))
    dt = 0.5 / 3000
    w = ti.ricker(250.0, dt).w32
    srcs = [(256, 256, 256), (5, 7, 9), (500, 250, 60), (130, 480, 400), (255, 255, 320)]
    sims = [tcm.Simulation(shapes, 1.0, dt, [lay] * 5, np.float32(1e-5), np.float32(1e-6), three_pass_update=tp)
            for tp in (False, True)]
    for sim in sims:
        for i, xyz in enumerate(srcs):
            sim.add_source(xyz, (1.0 - 0.3 * i) * w, shot=i)
    keys = ("step", "active_blocks", "activations", "retirements", "cell_updates", "peak_active_blocks")
    for k in range(150):
        for sim in sims:
            sim.step(1)
        a, b = sims[0].stats(), sims[1].stats()
        for key in keys:
            assert a[key] == b[key], (k, key)
    assert sims[0].stats()["active_blocks"] > 1000
    assert sims[0].check() == 0
    for shot in range(5):
        assert values_equal(sims[0].read(0, shot=shot), sims[1].read(0, shot=shot))
        assert values_equal(sims[0].read(1, shot=shot), sims[1].read(1, shot=shot))
    for sim in sims:
        sim.close()


@pytest.mark.parametrize("pool", ["key", "capped"])
def test_lattice_records_equal_c2_planes(pool):
    """Lattice media: blocks inside one lattice cell (spacing 8 or 16) and
    inside the domain take their C2 from the cell's 8 corners in the
    stencil; the fields and the work equal those of the same runs reading
    every C2 plane, bit for bit, and equal the CPU TCM on the dense media.
    A batch with spacings 8, 16 and 4 (no records) and ragged edges, a pool
    of one slot per key (records written when the pool is made) or a capped
    pool (written at activation), and single shots with dx = 2 (a power of
    two) and dx = 3."""
    announce(f"lattice records vs C2 planes ({pool} pool)")
    shapes = [(100, 90, 70), (64, 72, 64), (72, 40, 50)]
    lats = [ti.lognormal_lattice(sh, seed=70 + i, sigma=10.0, spacing=sp)
            for i, (sh, sp) in enumerate(zip(shapes, (8, 16, 4)))]
    dt = 0.5 / 4500.0
    w = ti.ricker(300.0, dt).w32
    srcs = [(50, 45, 35), (20, 30, 40), (36, 20, 25)]
    cap = 0 if pool == "key" else 3000      # capped: below the batch's 3840 keys, above its peak
    runs = []
    for planes in (False, True):
        sim = tcm.Simulation(shapes, 1.0, dt, lats, np.float32(1e-7), np.float32(1e-8), c2_planes=planes,
                             pool_bytes=cap * 6144)
        for i, xyz in enumerate(srcs):
            sim.add_source(xyz, w, shot=i)
        sim.step(160)
        assert sim.check() == 0
        runs.append(([sim.read(k, shot=i) for i in range(3) for k in (0, 1)], sim.stats()))
        sim.close()
    (fa, sa), (fb, sb) = runs
    assert all(values_equal(x, y) for x, y in zip(fa, fb))
    for key in ("active_blocks", "activations", "retirements", "cell_updates", "peak_active_blocks"):
        assert sa[key] == sb[key], key
    assert sa["active_blocks"] > 100
    # shot 1 against the CPU TCM on its dense media
    c1 = ti.lattice_to_dense(lats[1], shapes[1])
    t = oracle.TCM(c1, dt, 1.0, np.float32(1e-7), np.float32(1e-8))
    t.add_source(srcs[1], w)
    assert t.step(160) == 0
    assert values_equal(fa[2], t.read(0)) and values_equal(fa[3], t.read(1))
    # node spacings that are and are not powers of two
    for dx in (2.0, 3.0):
        out = []
        for planes in (False, True):
            sim = tcm.Simulation(shapes[0], dx, dt * dx, lats[0], 0.0, 0.0, c2_planes=planes,
                                 pool_bytes=(0 if pool == "key" else 2000) * 6144)
            sim.add_source(srcs[0], w)
            sim.step(60)
            out.append((sim.read(0), sim.read(1)))
            sim.close()
        assert values_equal(out[0][0], out[1][0]) and values_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("pool", ["key", "capped"])
def test_lattice_records_survive_restore_and_follow_set_media(pool):
    """Lattice records with checkpoints and new media: a snapshot restored
    mid-run repeats the run bit for bit (a capped pool rewrites the records
    of the restored blocks), and after tcm_set_media the run equals a fresh
    handle on the new media that reads every C2 plane."""
    announce(f"lattice records: restore and set_media ({pool} pool)")
    shape = (80, 72, 64)
    a = ti.lognormal_lattice(shape, seed=90, sigma=10.0, spacing=8)
    b = ti.lognormal_lattice(shape, seed=91, sigma=10.0, spacing=8)
    dt = 0.5 / 4500.0
    w = ti.ricker(300.0, dt).w32
    src = (40, 36, 30)
    kw = dict(pool_bytes=(0 if pool == "key" else 900) * 6144)
    sim = tcm.Simulation(shape, 1.0, dt, a, np.float32(1e-7), np.float32(1e-8), **kw)
    sim.add_source(src, w)
    sim.step(60)
    snap = sim.snapshot()
    sim.step(40)
    ref = (sim.read(0), sim.read(1), sim.stats()["cell_updates"])
    assert sim.stats()["lattice_cell_updates"] > 0
    sim.restore(snap)
    sim.step(40)
    assert values_equal(sim.read(0), ref[0]) and values_equal(sim.read(1), ref[1])
    assert sim.stats()["cell_updates"] == ref[2]
    snap.close()
    sim.set_media(b)
    sim.add_source(src, w)
    sim.step(70)
    fresh = tcm.Simulation(shape, 1.0, dt, b, np.float32(1e-7), np.float32(1e-8), c2_planes=True, **kw)
    fresh.add_source(src, w)
    fresh.step(70)
    assert values_equal(sim.read(0), fresh.read(0)) and values_equal(sim.read(1), fresh.read(1))
    assert sim.stats()["cell_updates"] == fresh.stats()["cell_updates"]
    assert sim.stats()["lattice_cell_updates"] > 0 and fresh.stats()["lattice_cell_updates"] == 0
    sim.close()
    fresh.close()


def block_key(shape, bx, by, bz):
    """Key of block (bx, by, bz): blocks in 4x4x4 tiles, tiles x-fastest,
    blocks inside a tile x-fastest (one pool slot per key when the pool holds
    every key)."""
    tx, ty = -(-shape[0] // 32), -(-shape[1] // 32)
    tile = ((bz >> 2) * ty + (by >> 2)) * tx + (bx >> 2)
    return tile * 64 + ((bz & 3) << 4) + ((by & 3) << 2) + (bx & 3)


@pytest.mark.parametrize("path,interval,at", [("two-launch", 1, 10), ("three-pass", 1, 10),
                                              ("interval", 8, 10), ("interval", 8, 7)])
def test_nonfinite_value_stops_the_run(path, interval, at):
    """A NaN written into phi^n of an active block (through a caller-owned
    pool, one slot per key): the next step reports TCM_E_NONFINITE, completes
    with its old active set (the NaN and its six neighbours are in phi^{n+1}),
    and later steps do nothing; the tables stay consistent and a snapshot
    from before the write runs on as a clean run does."""
    import torch
    announce(f"non-finite field: {path} update, interval {interval}, NaN at step {at}")
    shape = (64, 48, 40)
    nkeys = 2 * 2 * 2 * 64
    c = ti.random_media(shape, seed=77, cmin=0.6, cmax=1.0)
    w = ti.ricker(0.12, 0.5).w32
    src = (20, 21, 19)
    pool = torch.zeros(nkeys * 1536, dtype=torch.float32, device="cuda")
    sim = tcm.Simulation(shape, 1.0, 0.5, c, 1e-6, 1e-6, device_pool=pool, pool_bytes=nkeys * 6144,
                         three_pass_update=path == "three-pass", trigger_interval=interval)
    clean = tcm.Simulation(shape, 1.0, 0.5, c, 1e-6, 1e-6, three_pass_update=path == "three-pass",
                           trigger_interval=interval)
    for s in (sim, clean):
        s.add_source(src, w)
        s.step(at)
    snap = sim.snapshot()
    key = block_key(shape, src[0] // 8, src[1] // 8, src[2] // 8)
    local = ((src[2] % 8) * 8 + src[1] % 8) * 8 + src[0] % 8
    pool[((at & 1) * nkeys + key) * 512 + local] = float("nan")   # phi^at of the source node
    torch.cuda.synchronize()
    assert sim.step_status(5) == tcm.TCM_E_NONFINITE
    st = sim.stats()
    assert st["step"] == at + 1 and st["error"] == tcm.TCM_E_NONFINITE
    assert "not finite" in sim.last_error()
    phi = sim.read(0)
    bad = np.argwhere(np.isnan(phi))
    want = {(src[2], src[1], src[0])} | {(src[2] + dz, src[1] + dy, src[0] + dx) for dx, dy, dz in
                                         [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]}
    assert {tuple(int(v) for v in b) for b in bad} == want
    assert sim.check() == 0
    assert sim.step_status(1) == tcm.TCM_E_NONFINITE and sim.stats()["step"] == at + 1
    sim.restore(snap)
    assert sim.stats()["error"] == 0
    sim.step(6)
    clean.step(6)
    assert values_equal(sim.read(0), clean.read(0)) and values_equal(sim.read(1), clean.read(1))
    assert sim.stats()["active_blocks"] == clean.stats()["active_blocks"]


@pytest.mark.parametrize("engine,pool", [("blocks", "key"), ("blocks", "capped"), ("dense", "key")])
def test_set_media_equals_a_fresh_handle(engine, pool):
    """tcm_set_media on a handle that has run: the next run equals a handle
    created with the new media (fields and work), with a pool of one slot per
    key (C2 planes filled when the pool was made) or a capped pool; a
    snapshot from before the change is refused, speeds that break eq.(4)
    are refused and leave the old media in place, another media kind is
    refused."""
    announce(f"set_media ({engine}, {pool} pool)")
    shape = (40, 33, 27)
    a = ti.random_media(shape, seed=81, cmin=0.5, cmax=1.0)
    b = ti.random_media(shape, seed=82, cmin=0.4, cmax=0.9)
    w = ti.ricker(0.12, 0.5).w32
    src = (19, 16, 12)
    cap = 0 if pool == "key" else 60
    kw = dict(engine=engine, pool_bytes=cap * 6144)
    def run(sim, n):
        sim.add_source(src, w)
        sim.set_receivers([(3, 4, 5), (20, 16, 12)])
        sim.step(n)
        return sim.read(0), sim.read(1), sim.read_traces(), sim.stats()
    sim = tcm.Simulation(shape, 1.0, 0.5, a, 1e-4, 1e-5, **kw)
    run(sim, 30)
    snap = sim.snapshot()
    sim.set_media(b)
    assert sim.stats()["step"] == 0
    got = run(sim, 50)
    ref = run(tcm.Simulation(shape, 1.0, 0.5, b, 1e-4, 1e-5, **kw), 50)
    for x, y in zip(got[:3], ref[:3]):
        assert values_equal(x, y)
    for k in ("step", "active_blocks", "cell_updates", "activations", "retirements"):
        assert got[3][k] == ref[3][k], k
    with pytest.raises(tcm.TCMError):
        sim.restore(snap)
    with pytest.raises(tcm.TCMError) as e:
        sim.set_media(b * np.float32(2.0))          # cmax dt / dx = 0.9 > 1/sqrt(3)
    assert e.value.status == tcm.TCM_E_CFL
    with pytest.raises(tcm.TCMError):
        sim.set_media(ti.LayeredMedia(z_top=[0, 10], c_layer=[0.5, 0.9]))
    sim.reset()
    again = run(sim, 50)
    for x, y in zip(again[:3], ref[:3]):
        assert values_equal(x, y)
