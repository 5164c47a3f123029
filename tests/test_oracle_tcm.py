"""Pins of the CPU TCM oracle (O2).

* trigger = retire = 0 reproduces the dense grid exactly (the 7-point stencil
  moves information one node per step, so face triggering every step
  activates every cell that the dense solution makes nonzero);
* an infinite trigger level isolates the source cell: the result is the dense
  solution on that cell alone with zero ghosts;
* bookkeeping invariants of Table 1 (Cell2box / Box2cell bijection, every box
  either active or vacant, vacant boxes initialised); the activation rules
  themselves are pinned in test_oracle_rules.py;
* the result does not depend on the order in which boxes are stepped;
* a box cap fails deterministically and keeps the last complete step.
"""
import numpy as np
import pytest

import oracle
import tcm_inputs as ti
from conftest import values_equal


def _run_dense(c, dt, steps, sources, dtype, receivers=None):
    return oracle.dense_run(c, dt, 1.0, steps, dtype, sources=sources, receivers=receivers)


def test_tau0_equals_dense_c1():
    w = ti.c1()
    src = [(w.source, w.wavelet.w32)]
    phi, prev, tr = _run_dense(w.c_dense, w.dt, w.steps, src, np.float32, receivers=[(40, 32, 32)])
    t = oracle.TCM(w.c_dense, w.dt, w.dx, 0.0, 0.0)
    assert t.add_source(w.source, w.wavelet.w32) == 0
    t.set_receivers([(40, 32, 32)])
    rc, ttr = t.step(w.steps, traces=True)
    assert rc == 0 and t.check() == 0
    assert values_equal(t.read(0), phi)
    assert values_equal(t.read(1), prev)
    assert values_equal(ttr, tr)
    st = t.stats()
    assert st["step"] == 100 and st["active"] == 512   # the front fills the 64^3 grid


@pytest.mark.parametrize("dtype,block", [(np.float32, 8), (np.float64, 8), (np.float32, 4),
                                         (np.float32, 5)])
def test_tau0_equals_dense_ragged_heterogeneous(dtype, block):
    """Grid edges that are not multiples of the cell edge, random media,
    one source on a cell corner and one on the domain edge."""
    shape = (37, 29, 21)
    c = ti.random_media(shape, seed=7, cmin=0.3, cmax=1.0)
    dt = 0.55
    wa = ti.ricker(0.12, dt).w32
    wb = -0.5 * ti.ricker(0.2, dt).w32
    srcs = [((16, 8, 8), wa), ((36, 0, 20), wb)]
    phi, prev, _ = _run_dense(c, dt, 140, srcs, dtype)
    t = oracle.TCM(c, dt, 1.0, 0.0, 0.0, block=block, dtype=dtype)
    for xyz, w in srcs:
        assert t.add_source(xyz, w) == 0
    for k in range(7):
        assert t.step(20) == 0
        assert t.check() == 0
    assert values_equal(t.read(0), phi)
    assert values_equal(t.read(1), prev)


def test_infinite_trigger_isolates_source_cell():
    """With thresholds above any field value only the pinned source cell runs;
    it evolves as the dense grid restricted to that cell (zero ghosts), and is
    unboxed once the source has no samples left."""
    shape = (32, 32, 32)
    c = np.ones(shape[::-1], np.float32)
    w = ti.ricker(0.15, 0.5).w32
    big = np.float32(1e30)
    t = oracle.TCM(c, 0.5, 1.0, big, big)
    t.add_source((13, 10, 9), w)            # cell (1,1,1), local (5,2,1)
    ns = w.size
    assert t.step(ns - 1) == 0
    alone, _, _ = _run_dense(np.ones((8, 8, 8), np.float32), 0.5, ns - 1,
                             [((5, 2, 1), w)], np.float32)
    out = t.read(0)
    assert values_equal(out[8:16, 8:16, 8:16], alone)
    out[8:16, 8:16, 8:16] = 0
    assert not out.any()
    assert t.stats()["active"] == 1
    assert t.step(1) == 0                    # last sample inserted; nothing is kept
    assert t.stats()["active"] == 0
    assert not t.read(0).any()
    assert t.check() == 0


def test_invariants_random_thresholds():
    """Table 1 bookkeeping stays consistent over uneven step chunks at
    thresholds above zero (the activation rules themselves are checked step by
    step in test_oracle_rules.py)."""
    rng = np.random.default_rng(9)
    shape = (40, 36, 30)
    c = ti.random_media(shape, seed=9, cmin=0.4, cmax=1.0)
    dt = 0.5
    w = ti.ricker(0.12, dt).w32
    trig, ret = np.float32(3e-4), np.float32(5e-5)
    t = oracle.TCM(c, dt, 1.0, trig, ret)
    t.add_source((20, 18, 15), w)
    for k in range(25):
        assert t.step(int(rng.integers(1, 6))) == 0
        assert t.check() == 0
    st = t.stats()
    assert 0 < st["active"] <= st["peak_active"] <= st["boxes"]
    assert st["activations"] - st["retirements"] == st["active"]


def test_processing_order_does_not_matter():
    w = ti.c1(steps=70)
    res = []
    for seed in (0, 7, 12345):
        t = oracle.TCM(w.c_dense, w.dt, 1.0, np.float32(1e-6), np.float32(1e-7))
        t.add_source(w.source, w.wavelet.w32)
        assert t.step(w.steps, order_seed=seed) == 0
        res.append((t.read(0), t.read(1)))
    for a, b in res[1:]:
        assert values_equal(a, res[0][0]) and values_equal(b, res[0][1])


def test_box_cap_fails_deterministically_and_keeps_last_step():
    w = ti.c1(steps=60)
    full = oracle.TCM(w.c_dense, w.dt, 1.0, 0.0, 0.0)
    full.add_source(w.source, w.wavelet.w32)
    counts = []
    for k in range(60):
        full.step(1)
        counts.append(full.stats()["active"])
    cap = 100
    fail_step = next(i for i, n in enumerate(counts) if n > cap)   # step index whose update overflows
    capped = oracle.TCM(w.c_dense, w.dt, 1.0, 0.0, 0.0, cap=cap)
    capped.add_source(w.source, w.wavelet.w32)
    rc = capped.step(60)
    assert rc == oracle.TCM.E_POOL
    st = capped.stats()
    assert st["step"] == fail_step + 1 and st["error"] == -3
    assert st["active"] == counts[fail_step - 1]
    assert capped.check() == 0
    # the kept level equals the dense field at that step
    phi, _, _ = _run_dense(w.c_dense, w.dt, fail_step + 1, [(w.source, w.wavelet.w32)], np.float32)
    assert values_equal(capped.read(0), phi)
    assert capped.step(5) == oracle.TCM.E_POOL and capped.stats()["step"] == fail_step + 1


def test_threshold_error_is_ordered_and_bounded():
    """Raising the trigger level lowers the work and raises the error against
    FP64 dense; the error stays within the stated bounds (C1 shape, retire =
    trigger / 10).  Below ~1e-7 of the peak the truncation is under the FP32
    rounding noise, so only a 2x band around the tau = 0 error is asserted."""
    w = ti.c1()
    ref, _, _ = _run_dense(w.c_dense, w.dt, w.steps, [(w.source, w.wavelet.w32.astype(np.float64))],
                           np.float64)
    nref = np.linalg.norm(ref)
    errs, work = {}, {}
    rels = (0.0, 1e-8, 1e-6, 1e-5, 1e-4)
    for rel in rels:
        t = oracle.TCM(w.c_dense, w.dt, 1.0, np.float32(rel * w.wavelet.peak),
                       np.float32(rel * w.wavelet.peak / 10))
        t.add_source(w.source, w.wavelet.w32)
        assert t.step(w.steps) == 0
        errs[rel] = np.linalg.norm(t.read(0).astype(np.float64) - ref) / nref
        work[rel] = t.stats()["updates"]
    assert errs[0.0] < 1e-6
    assert errs[1e-8] < 2 * errs[0.0]
    assert errs[1e-6] < 5e-5 and errs[1e-5] < 5e-4 and errs[1e-4] < 5e-3
    assert errs[1e-6] < errs[1e-5] < errs[1e-4]
    assert all(work[a] > work[b] for a, b in zip(rels, rels[1:]))


def test_shutdown_decay_total_attenuation_eq6():
    """With C2 = 0 a field with phi^n = phi^{n-1} is stationary; once its cell
    stops qualifying, n decay steps scale it by alpha each (A = alpha^n,
    eq.(6)), then the cell is unboxed."""
    c = np.ones((16, 16, 16), np.float32)
    n, alpha = 5, np.float32(0.5)
    t = oracle.TCM(c, 0.0, 1.0, np.float32(2.0), np.float32(2.0), shutdown_steps=n,
                   shutdown_alpha=alpha)
    t.add_source((3, 3, 3), np.array([1.0, -1.0], np.float32))
    vals = []
    for k in range(8):
        assert t.step(1) == 0
        vals.append(float(t.read(0)[3, 3, 3]))
    assert vals[:2] == [1.0, 0.5]
    assert vals[1:6] == [0.5 ** j for j in range(1, 6)]
    assert vals[5] == oracle.decay_total(0.5, n)
    assert vals[6] == 0.0 and t.stats()["active"] == 0 and t.check() == 0


def test_shutdown_decay_matches_explicit_emulation():
    """Isolated source cell (thresholds above every value): after the last
    sample it decays for n steps; emulate with the dense oracle on the cell
    alone plus explicit alpha scalings of both levels."""
    shape = (24, 24, 24)
    c = np.ones(shape[::-1], np.float32)
    w = ti.ricker(0.15, 0.5).w32
    big = np.float32(1e30)
    n, alpha = 7, np.float32(0.8)
    t = oracle.TCM(c, 0.5, 1.0, big, big, shutdown_steps=n, shutdown_alpha=alpha)
    t.add_source((13, 10, 9), w)
    alone = np.ones((8, 8, 8), np.float32)
    phi = np.zeros((8, 8, 8), np.float32)
    prev = np.zeros((8, 8, 8), np.float32)
    ns = w.size
    for k in range(ns + n + 2):
        assert t.step(1) == 0
        phi, prev, _ = oracle.dense_run(alone, 0.5, 1.0, 1, np.float32, phi=phi, phi_prev=prev,
                                        step0=k, sources=[((5, 2, 1), w)])
        if ns - 1 <= k < ns - 1 + n:          # cell no longer pinned: decay steps
            phi = phi * alpha
            prev = prev * alpha
        if k == ns - 1 + n:                   # shutdown finished: unboxed
            phi[:] = 0
            prev[:] = 0
        out = t.read(0)
        assert values_equal(out[8:16, 8:16, 8:16], phi), k
    assert t.stats()["active"] == 0 and t.check() == 0


def test_adaptive_levels_follow_domain_maximum():
    """Table 1 Trig_level relative to the domain maximum: the levels of each
    update are rel * max|phi^{n+1}| (the cell holding the maximum is kept)."""
    w = ti.c1(steps=80)
    rt, rr = np.float32(1e-3), np.float32(1e-4)
    t = oracle.TCM(w.c_dense, w.dt, 1.0, 0.0, 0.0, trigger_rel=rt, retire_rel=rr)
    t.add_source(w.source, w.wavelet.w32)
    work = []
    for k in range(80):
        assert t.step(1) == 0
        m = np.float32(np.max(np.abs(t.read(0))))
        trig, ret = t.levels()
        assert trig == float(rt * m) and ret == float(rr * m), k
        work.append(t.stats()["updates"])
    fixed = oracle.TCM(w.c_dense, w.dt, 1.0, 0.0, 0.0)
    fixed.add_source(w.source, w.wavelet.w32)
    fixed.step(80)
    assert work[-1] < fixed.stats()["updates"]
    zero = oracle.TCM(w.c_dense, w.dt, 1.0, 0.0, 0.0, trigger_rel=0.0, retire_rel=0.0)
    zero.add_source(w.source, w.wavelet.w32)
    zero.step(80)
    assert values_equal(zero.read(0), fixed.read(0))


@pytest.mark.parametrize("k", [2, 5, 8])
def test_update_interval_with_diagonal_lookahead_is_exact_at_tau0(k):
    """Activation every k <= 8 steps with the 26-cell neighbourhood keeps the
    threshold-0 TCM equal to the dense grid (values move one node per step);
    eq.(5) with a cell length of 8 nodes gives k = 8 at Courant 0.5."""
    assert oracle.update_interval(1.0, 8.0, 1.0, 0.5) == 8.0
    shape = (37, 29, 21)
    c = ti.random_media(shape, seed=7, cmin=0.3, cmax=1.0)
    dt = 0.55
    srcs = [((16, 8, 8), ti.ricker(0.12, dt).w32), ((36, 0, 20), -0.5 * ti.ricker(0.2, dt).w32)]
    phi, prev, _ = _run_dense(c, dt, 97, srcs, np.float32)
    t = oracle.TCM(c, dt, 1.0, 0.0, 0.0, interval=k)
    for xyz, w in srcs:
        t.add_source(xyz, w)
    for chunk in (13, 40, 44):
        assert t.step(chunk) == 0 and t.check() == 0
    assert values_equal(t.read(0), phi) and values_equal(t.read(1), prev)


def test_update_interval_rejects_more_than_a_cell():
    w = ti.c1()
    with pytest.raises(ValueError):
        oracle.TCM(w.c_dense, w.dt, 1.0, interval=9)
