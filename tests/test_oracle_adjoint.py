"""Pins of the FP64 adjoint oracle (O3) against the forward model (O1):
central finite differences of a receiver misfit, a directional-derivative
(dot-product) test with random residuals, and independence from the
checkpoint interval."""
import numpy as np
import pytest

import oracle
import tcm_inputs as ti


def _setup(seed=1):
    rng = np.random.default_rng(seed)
    shape = (10, 10, 10)
    c = 0.8 + 0.2 * ti.lattice_to_dense(ti.lognormal_lattice(shape, seed=seed, sigma=3.0, spacing=2,
                                                             cmin=0.1, cmax=10.0), shape)
    c = (c / c.max()).astype(np.float64)
    dt = 0.5
    w = ti.ricker(0.15, dt).w64
    src = [((3, 4, 5), w)]
    rec = [(7, 6, 5), (2, 8, 7), (5, 5, 8)]
    return rng, c, dt, src, rec


def _traces(c, dt, src, rec, nt):
    return oracle.dense_run(c, dt, 1.0, nt, np.float64, sources=src, receivers=rec)[2]


def test_adjoint_matches_central_differences():
    rng, c, dt, src, rec = _setup()
    nt = 40
    c_true = c * (1.0 + 0.05 * rng.standard_normal(c.shape))
    d = _traces(c_true, dt, src, rec, nt)
    J = lambda cc: 0.5 * np.sum((_traces(cc, dt, src, rec, nt) - d) ** 2)
    resid = _traces(c, dt, src, rec, nt) - d
    g = oracle.adjoint_f64(c, dt, 1.0, src, rec, resid, ckpt=7)
    cells = [(4, 4, 4), (5, 3, 6), (3, 5, 5), (6, 6, 4)]       # (x, y, z)
    for (x, y, z) in cells:
        h = 1e-5 * c[z, y, x]
        cp, cm = c.copy(), c.copy()
        cp[z, y, x] += h
        cm[z, y, x] -= h
        fd = (J(cp) - J(cm)) / (2 * h)
        assert abs(g[z, y, x]) > 1e-8
        assert abs(fd - g[z, y, x]) <= 1e-6 * abs(g[z, y, x]) + 1e-14


def test_adjoint_dot_product_with_random_residual():
    rng, c, dt, src, rec = _setup(2)
    nt = 35
    r = rng.standard_normal((nt, len(rec)))
    g = oracle.adjoint_f64(c, dt, 1.0, src, rec, r, ckpt=10)
    dc = rng.standard_normal(c.shape)
    h = 1e-6
    dtr = (_traces(c + h * dc, dt, src, rec, nt) - _traces(c - h * dc, dt, src, rec, nt)) / (2 * h)
    lhs = np.sum(dtr * r)
    rhs = np.sum(dc * g)
    assert abs(lhs - rhs) <= 1e-7 * abs(rhs)


def test_adjoint_independent_of_checkpoint_interval():
    rng, c, dt, src, rec = _setup(3)
    nt = 30
    r = rng.standard_normal((nt, len(rec)))
    g1 = oracle.adjoint_f64(c, dt, 1.0, src, rec, r, ckpt=1)
    g7 = oracle.adjoint_f64(c, dt, 1.0, src, rec, r, ckpt=7)
    g30 = oracle.adjoint_f64(c, dt, 1.0, src, rec, r, ckpt=30)
    s = np.max(np.abs(g30))
    assert np.max(np.abs(g1 - g30)) < 1e-13 * s and np.max(np.abs(g7 - g30)) < 1e-13 * s


def test_adjoint_zero_speed_cells_have_zero_gradient():
    rng, c, dt, src, rec = _setup(4)
    c = c.copy()
    c[5, 5, 5] = 0.0
    r = rng.standard_normal((20, len(rec)))
    g = oracle.adjoint_f64(c, dt, 1.0, src, rec, r, ckpt=5)
    assert g[5, 5, 5] == 0.0 and np.isfinite(g).all()
