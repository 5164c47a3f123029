"""Pins of the CPU TCM oracle's activation rules ("Updating active cells",
items 1-4, update after every step, no shutdown).

* After every step the oracle's active cells equal the rules evaluated
  test-side (tests/activation_rules.py) from the previous active set, phi^n
  and phi^{n+1}; phi^{n+1} comes from one step of the dense oracle on the
  previous fields, and the kept cells hold exactly those values.
* At threshold 0 the active set is derived from the dense oracle's own
  fields alone.
* Closed forms with C2 = 0 (a field that changes only at its source node)
  pin the two choices the paper leaves open: a cell whose new level is zero
  but whose current level is not keeps running (its next level is minus the
  current one), and both comparisons are strict.
"""
import numpy as np
import pytest

import oracle
import tcm_inputs as ti
from activation_rules import cells_shape, next_active, node_mask
from conftest import values_equal


def _pinned(sources, n, B):
    """Cells of sources that still insert a sample at step n + 1."""
    out = []
    for (x, y, z), w, t0 in sources:
        if n + 1 < t0 + len(w):
            out.append((z // B, y // B, x // B))
    return out


def _check_steps(c, dt, t, sources, nsteps, B, dtype, levels=None):
    """Step the oracle one step at a time and check every update against the
    rules.  ``sources``: ((x, y, z), w, start step) already added to t.
    ``levels(t)`` gives the (trigger, retire) the update used; by default
    the constant levels of the run."""
    shape = c.shape
    for _ in range(nsteps):
        n = t.stats()["step"]
        act = t.triggered().astype(bool)
        cur, prv = t.read(0), t.read(1)
        full, _, _ = oracle.dense_run(c, dt, 1.0, 1, dtype, phi=cur, phi_prev=prv, step0=n,
                                      sources=sources)
        amask = node_mask(act, shape, B)
        new = np.where(amask, full, dtype(0))
        assert t.step(1) == 0
        trig, ret = levels(t)
        want = next_active(new, cur, act, trig, ret, _pinned(sources, n, B), B)
        got = t.triggered().astype(bool)
        assert np.array_equal(got, want), f"step {n}: active cells differ from the rules"
        kept = node_mask(act & want, shape, B)
        assert values_equal(t.read(0), np.where(kept, new, dtype(0))), n
        assert values_equal(t.read(1), np.where(kept, cur, dtype(0))), n


@pytest.mark.parametrize("case", ["hysteresis", "single_level", "retiring", "tau0_ragged", "adaptive",
                                  "f64"])
def test_activation_update_follows_the_rules_every_step(case):
    """Random media in a small box (waves reflect, nothing is released), and
    a homogeneous box at a single level where the pulse leaves cells behind
    it (cells are released, some only one step after their new level fell
    below the level)."""
    B = 8
    dtype = np.float64 if case == "f64" else np.float32
    shape = {"tau0_ragged": (38, 33, 27), "retiring": (56, 52, 48)}.get(case, (40, 36, 30))
    c = ti.random_media(shape, seed=9, cmin=0.4, cmax=1.0)
    if case == "retiring":
        c = np.ones_like(c)
    dt = 0.5
    w = ti.ricker(0.15 if case == "retiring" else 0.12, dt).w32.astype(dtype)
    peak = float(np.max(np.abs(w)))
    kw = {}
    if case == "retiring":
        trig = ret = 3e-3 * peak
    elif case == "hysteresis" or case == "f64":
        trig, ret = 3e-4 * peak, 5e-5 * peak
    elif case == "single_level":
        trig = ret = 1e-4 * peak
    elif case == "tau0_ragged":
        trig = ret = 0.0
    else:
        trig, ret = 0.0, 0.0
        kw = dict(trigger_rel=1e-3, retire_rel=2e-4)
    t = oracle.TCM(c, dt, 1.0, dtype(trig), dtype(ret), block=B, dtype=dtype, **kw)
    sources = [((20, 18, 15), w, 0)]
    if case == "tau0_ragged":
        sources.append(((37, 0, 26), -0.5 * w, 0))      # on the ragged domain edge
    for xyz, ws, _ in sources:
        assert t.add_source(xyz, ws) == 0
    levels = (lambda tt: tt.levels()) if case == "adaptive" else (lambda tt: (trig, ret))
    _check_steps(c, dt, t, sources, 90, B, dtype, levels)
    # a source added mid-run boxes its cell at once and pins it
    n = t.stats()["step"]
    sources.append(((3, 30, 4), w, n))
    assert t.add_source((3, 30, 4), w) == 0
    assert t.triggered()[0, 3, 0] == 1
    _check_steps(c, dt, t, sources, 40, B, dtype, levels)
    assert t.check() == 0
    if case == "retiring":
        assert t.stats()["retirements"] > 0


def test_threshold0_active_set_follows_the_dense_field():
    """At threshold 0 the TCM equals the dense grid, so the active cells of
    every step follow from the dense fields: the cells holding a nonzero value
    of phi^{n+1} or phi^n, those across a face with a nonzero phi^{n+1}, and
    the pinned source cell."""
    B = 8
    shape = (41, 35, 29)
    c = ti.random_media(shape, seed=21, cmin=0.3, cmax=1.0)
    dt = 0.55
    w = ti.ricker(0.15, dt).w32
    src = (9, 24, 16)
    t = oracle.TCM(c, dt, 1.0, 0.0, 0.0, block=B)
    assert t.add_source(src, w) == 0
    cur = np.zeros_like(c)
    prv = np.zeros_like(c)
    act = np.zeros(cells_shape(c.shape, B), bool)
    act[src[2] // B, src[1] // B, src[0] // B] = True
    assert np.array_equal(t.triggered().astype(bool), act)
    for n in range(80):
        new, _, _ = oracle.dense_run(c, dt, 1.0, 1, np.float32, phi=cur, phi_prev=prv, step0=n,
                                     sources=[(src, w)])
        pins = [(src[2] // B, src[1] // B, src[0] // B)] if n + 1 < w.size else []
        act = next_active(new, cur, np.ones_like(act), 0.0, 0.0, pins, B)
        prv, cur = cur, new
        assert t.step(1) == 0
        assert np.array_equal(t.triggered().astype(bool), act), n
        assert values_equal(t.read(0), cur) and values_equal(t.read(1), prv), n
    assert act.sum() > 20


def test_cell_keeps_running_while_its_current_level_is_nonzero():
    """C2 = 0: the update is u^{n+1} = 2 u^n - u^{n-1} + w[n] at the source
    node and zero elsewhere.  With w = (a, -2a) the source node takes
    u^1 = a, u^2 = 0 and then u^n = (2 - n) a.  At step 1 the cell's new level
    is all zero but its current level is not: it must stay active (and then
    grow as the closed form says), both at threshold 0 and with a keep level
    below |a|; an interior node triggers no face."""
    a = np.float32(0.25)
    c = np.zeros((16, 16, 16), np.float32)
    w = np.array([a, -2 * a], np.float32)
    for trig, ret in ((0.0, 0.0), (1e30, 0.125)):
        t = oracle.TCM(c, 0.5, 1.0, np.float32(trig), np.float32(ret))
        assert t.add_source((3, 4, 5), w) == 0
        for n in range(1, 12):
            assert t.step(1) == 0
            u = t.read(0)
            assert u[5, 4, 3] == (a if n == 1 else (2 - n) * a), (trig, n)
            u[5, 4, 3] = 0
            assert not u.any()
            assert t.stats()["active"] == 1, (trig, n)
        dense, _, _ = oracle.dense_run(c, 0.5, 1.0, 11, np.float32, sources=[((3, 4, 5), w)])
        assert values_equal(t.read(0), dense)


@pytest.mark.parametrize("which", ["trigger", "retire"])
def test_comparisons_are_strict_at_exact_levels(which):
    """C2 = 0 and w = (a, -a): the source node holds a from step 1 on, on the
    cell's +x face.  With the level exactly a nothing exceeds it: the cell
    across the face is never activated, and the source cell is released once
    its samples end.  One ulp below a, the face triggers the neighbour
    (trigger) or the cell is kept (retire)."""
    a = np.float32(0.25)
    below = np.nextafter(a, np.float32(0))
    c = np.zeros((24, 16, 16), np.float32)
    w = np.array([a, -a], np.float32)
    for lvl in (a, below):
        trig, ret = (lvl, np.float32(0.0)) if which == "trigger" else (np.float32(1e30), lvl)
        t = oracle.TCM(c, 0.5, 1.0, trig, ret)
        assert t.add_source((7, 3, 3), w) == 0          # x = 7: the +x face of cell (0, 0, 0)
        actives = []
        for n in range(6):
            assert t.step(1) == 0
            actives.append(t.triggered().astype(bool).copy())
            assert t.read(0)[3, 3, 7] in (a, 0)
        if which == "trigger":
            # retire 0: the source cell stays (its value a > 0); its +x neighbour only if a > trigger
            assert all(m[0, 0, 0] for m in actives)
            assert all(m[0, 0, 1] == (lvl < a) for m in actives)
        else:
            # pinned for step 0 only; then kept only if a > retire
            assert actives[0][0, 0, 0]
            assert all(m[0, 0, 0] == (lvl < a) for m in actives[1:])
            assert not any(m[0, 0, 1] for m in actives)
