"""Batched shots over one shared pool: each shot must be bit-exact to its own
single-shot run and to the CPU oracle (the shots never interact)."""
import numpy as np
import pytest

import oracle
import tcm_inputs as ti
from conftest import values_equal

pytestmark = pytest.mark.gpu
tcm = pytest.importorskip("paper_1702_00216_amd")


def announce(msg):
    print(f"\n[case] {msg}", flush=True)


def make_shots(n=5, seed=4, lo=20, hi=56):
    rng = np.random.default_rng(seed)
    shots = []
    for i in range(n):
        shape = tuple(int(v) for v in rng.integers(lo, hi + 1, size=3))
        lat = ti.lognormal_lattice(shape, seed=100 + i, sigma=5.0, spacing=4)
        src = tuple(int(rng.integers(2, e - 2)) for e in shape)
        shots.append((shape, lat, src))
    return shots


@pytest.mark.parametrize("trig", [0.0, 3e-4])
def test_batch_equals_single_shots_and_oracle(trig):
    announce(f"batch of 5 shots, trigger {trig}")
    dt = 0.5 / 4500
    w = ti.ricker(300.0, dt).w32
    shots = make_shots()
    trig = np.float32(trig)
    ret = np.float32(trig / 4)
    b = tcm.Simulation([s[0] for s in shots], 1.0, dt, [s[1] for s in shots], trig, ret)
    for i, (shape, lat, src) in enumerate(shots):
        b.add_source(src, w, shot=i)
    rec = [(1, 2, 3), (5, 5, 5), (0, 0, 0)]
    b.set_receivers(rec, shots=[0, 2, 4])
    b.step(75)
    traces = b.read_traces()
    for i, (shape, lat, src) in enumerate(shots):
        single = tcm.Simulation(shape, 1.0, dt, lat, trig, ret)
        single.add_source(src, w)
        single.step(75)
        assert values_equal(b.read(0, shot=i), single.read(0)), i
        assert values_equal(b.read(1, shot=i), single.read(1)), i
        cd = ti.lattice_to_dense(lat, shape)
        t = oracle.TCM(cd, dt, 1.0, trig, ret)
        t.add_source(src, w)
        t.step(75)
        assert values_equal(b.read(0, shot=i), t.read(0)), i
        if trig == 0:
            phi, _, _ = oracle.dense_run(cd, dt, 1.0, 75, np.float32, sources=[(src, w)])
            assert values_equal(b.read(0, shot=i), phi), i
    for r, (xyz, s) in enumerate(zip(rec, [0, 2, 4])):
        shape, lat, src = shots[s]
        cd = ti.lattice_to_dense(lat, shape)
        t = oracle.TCM(cd, dt, 1.0, trig, ret)
        t.add_source(src, w)
        t.set_receivers([xyz])
        _, tr = t.step(75, traces=True)
        assert values_equal(traces[:, r], tr[:, 0])


def test_batch_shared_pool_overflow_is_reported():
    announce("batch pool overflow")
    dt = 0.5 / 4500
    w = ti.ricker(300.0, dt).w32
    shots = make_shots(3, seed=9)
    b = tcm.Simulation([s[0] for s in shots], 1.0, dt, [s[1] for s in shots], pool_bytes=40 * 6144)
    for i, (shape, lat, src) in enumerate(shots):
        b.add_source(src, w, shot=i)
    with pytest.raises(tcm.TCMError) as ei:
        b.step(200)
    assert ei.value.status == -3
    st = b.stats()
    assert st["error"] == -3 and st["active_blocks"] <= 40


def test_autotune_keeps_state_and_results(tmp_path):
    announce("autotune: state unchanged, results unchanged, cache")
    dt = 0.5 / 4500
    w = ti.ricker(300.0, dt).w32
    shots = make_shots(4, seed=21)
    def fresh():
        b = tcm.Simulation([s[0] for s in shots], 1.0, dt, [s[1] for s in shots], 1e-4, 1e-5)
        for i, (shape, lat, src) in enumerate(shots):
            b.add_source(src, w, shot=i)
        return b
    a = fresh()
    a.step(40)
    before = [a.read(0, shot=i) for i in range(4)], a.stats()
    res = a.autotune(probe_steps=8)
    after = [a.read(0, shot=i) for i in range(4)], a.stats()
    for x, y in zip(before[0], after[0]):
        assert values_equal(x, y)
    for k in ("step", "active_blocks", "cell_updates", "activations", "retirements"):
        assert before[1][k] == after[1][k], k
    assert res["candidates"] and (res["blocks_per_wg"], res["blocks_per_wave"], res["wg_per_cu"],
                                  res["graph_steps"]) in [(c[0], c[1], c[2], c[3]) for c in res["candidates"]]
    # every tile, with one and (tiles of 4 and 8) two blocks per wave
    assert {(c[0], c[1]) for c in res["candidates"]} == {(2, 1), (4, 1), (8, 1), (4, 2), (8, 2)}
    a.step(60)
    ref = fresh()
    ref.step(100)
    for i in range(4):
        assert values_equal(a.read(0, shot=i), ref.read(0, shot=i))
    cache = str(tmp_path / "tune.json")
    r1 = ref.autotune(probe_steps=4, cache=cache, key="gfx950/test")
    r2 = fresh().autotune(probe_steps=4, cache=cache, key="gfx950/test")
    assert not r1["cached"] and r2["cached"] and r2["wg_per_cu"] == r1["wg_per_cu"]
    assert r2["blocks_per_wg"] == r1["blocks_per_wg"] and r2["blocks_per_wave"] == r1["blocks_per_wave"]
    with pytest.raises(tcm.TCMError):
        ref.set_launch(0, 16)


def test_autotune_run_keeps_state_and_picks_a_timed_family(tmp_path):
    """The whole-run tuner steps the run to probe three states and times every
    tile family over the whole run, then restores the state: the field,
    statistics and later results are those of an untuned run, and the shape
    it keeps is the family with the shortest whole run."""
    announce("autotune over a whole run")
    dt = 0.5 / 4500
    w = ti.ricker(300.0, dt).w32
    shots = make_shots(3, seed=23)
    def fresh():
        b = tcm.Simulation([s[0] for s in shots], 1.0, dt, [s[1] for s in shots], 1e-4, 1e-5)
        for i, (shape, lat, src) in enumerate(shots):
            b.add_source(src, w, shot=i)
        return b
    a = fresh()
    a.step(5)
    before = [a.read(0, shot=i) for i in range(3)], a.stats()
    res = a.autotune_run(48, probe_steps=4)
    after = [a.read(0, shot=i) for i in range(3)], a.stats()
    for x, y in zip(before[0], after[0]):
        assert values_equal(x, y)
    for k in ("step", "active_blocks", "cell_updates", "activations", "retirements"):
        assert before[1][k] == after[1][k], k
    fam = res["families"]
    assert len(fam) == 5 and all(v > 0 for v in fam.values())
    chosen = f"{res['blocks_per_wg']}x{res['blocks_per_wave']}@{res['wg_per_cu']}"
    assert fam[chosen] == min(fam.values())
    assert res["ms_per_step"] == pytest.approx(fam[chosen] / 48, abs=1e-4)
    a.step(60)
    ref = fresh()
    ref.step(65)
    for i in range(3):
        assert values_equal(a.read(0, shot=i), ref.read(0, shot=i))
    cache = str(tmp_path / "tune.json")
    r1 = fresh().autotune_run(16, probe_steps=2, cache=cache, key="gfx950/test/run")
    r2 = fresh().autotune_run(16, probe_steps=2, cache=cache, key="gfx950/test/run")
    assert not r1["cached"] and r2["cached"] and r2["families"] == r1["families"]


@pytest.mark.parametrize("seed", list(range(8)))
def test_random_batches_match_cpu_tcm_per_shot(seed):
    """Seeded random batches: 2-7 shots of random shapes, media and sources
    over one pool (auto or just above the summed peaks), random levels,
    update interval and workgroup tile (one or two blocks per wave); every
    shot equals the CPU TCM run on its own."""
    rng = np.random.default_rng(500 + seed)
    nshot = int(rng.integers(2, 8))
    dt = 0.55
    tr = float(rng.choice([0.0, 1e-4, 1e-3]))
    trig, ret = np.float32(tr), np.float32(tr * 0.3)
    interval = int(rng.choice([1, 1, 2, 8]))
    tile = int(rng.choice([2, 4, 8]))
    per_wave = 1 + seed % 2 if tile > 2 else 1          # not drawn: the other choices stay as they were
    steps = int(rng.integers(30, 120))
    shots = []
    for i in range(nshot):
        shape = tuple(int(v) for v in rng.integers(4, 48, size=3))
        c = ti.random_media(shape, seed=6000 + 10 * seed + i, cmin=0.3, cmax=1.0)
        src = tuple(int(rng.integers(0, e)) for e in shape)
        shots.append((shape, c, src, ti.ricker(float(rng.uniform(0.08, 0.2)), dt).w32))
    ref = []
    for shape, c, src, w in shots:
        t = oracle.TCM(c, dt, 1.0, trig, ret, interval=interval)
        t.add_source(src, w)
        assert t.step(steps) == 0
        ref.append(t)
    cap = 0
    if seed % 2:
        cap = max(64, sum(t.stats()["peak_active"] for t in ref) + int(rng.integers(0, 30)))
    announce(f"random batch {seed}: {nshot} shots, levels {tr:g}, k {interval}, tile {tile}x{per_wave}, "
             f"pool {cap or 'auto'}")
    b = tcm.Simulation([s[0] for s in shots], 1.0, dt, [s[1] for s in shots], trig, ret,
                       trigger_interval=interval, blocks_per_wg=tile, blocks_per_wave=per_wave,
                       pool_bytes=cap * 6144)
    for i, (shape, c, src, w) in enumerate(shots):
        b.add_source(src, w, shot=i)
    b.step(steps)
    tot = 0
    for i, t in enumerate(ref):
        assert values_equal(b.read(0, shot=i), t.read(0)), i
        assert values_equal(b.read(1, shot=i), t.read(1)), i
        tot += t.stats()["updates"]
    assert b.stats()["cell_updates"] == tot
