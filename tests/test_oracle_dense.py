"""Pins of the dense oracle (O1) against closed forms and conservation laws.

Each test would fail for a plausible slip in the oracle: a wrong time level,
a wrong or transposed neighbour index, a dropped Laplacian term, a wrong sign
or a misplaced C^2 coefficient.
"""
import math

import numpy as np
import pytest

import oracle
from conftest import values_equal


def _laplacian(u):
    """7-point Laplacian with zero ghosts (test-side definition of A = -L)."""
    p = np.pad(u, 1)
    return (p[1:-1, 1:-1, 2:] + p[1:-1, 1:-1, :-2] + p[1:-1, 2:, 1:-1] + p[1:-1, :-2, 1:-1]
            + p[2:, 1:-1, 1:-1] + p[:-2, 1:-1, 1:-1] - 6.0 * u)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_dalembert_1d_courant_one_is_exact(dtype):
    """Central differences at Courant 1 in 1-D reproduce u(i, n) = f(i - n) + g(i + n)
    exactly (Introduction, eq.(2)-(3) in one dimension)."""
    nx = 420
    f = np.zeros(nx)
    g = np.zeros(nx)
    f[118:123] = [1, 3, 7, 3, 1]          # right-moving, integer valued
    g[280:284] = [2, -5, 4, 1]            # left-moving
    shift = lambda a, k: np.roll(a, k)    # pulses stay far from the ends
    phi0 = f + g
    phim1 = shift(f, -1) + shift(g, 1)    # u(i, -1) = f(i + 1) + g(i - 1)
    c = np.ones((1, 1, nx))
    steps = 150
    phi, prev, _ = oracle.dense_run(c, 1.0, 1.0, steps, dtype, phi=phi0.reshape(1, 1, nx),
                                    phi_prev=phim1.reshape(1, 1, nx), ndim=1)
    expect = shift(f, steps) + shift(g, -steps)
    expect_prev = shift(f, steps - 1) + shift(g, -(steps - 1))
    assert values_equal(phi.ravel(), expect.astype(dtype))
    assert values_equal(prev.ravel(), expect_prev.astype(dtype))


def test_dalembert_1d_smooth_fp64():
    nx = 600
    i = np.arange(nx, dtype=np.float64)
    f = lambda x: np.exp(-((x - 200.0) / 12.0) ** 2)
    phi0 = f(i)
    phim1 = f(i + 1)
    c = np.ones((1, 1, nx))
    phi, _, _ = oracle.dense_run(c, 1.0, 1.0, 180, np.float64, phi=phi0.reshape(1, 1, nx),
                                 phi_prev=phim1.reshape(1, 1, nx), ndim=1)
    assert np.max(np.abs(phi.ravel() - f(i - 180))) < 1e-14


def _mode(shape, k):
    nx, ny, nz = shape
    x = np.arange(nx)[None, None, :]
    y = np.arange(ny)[None, :, None]
    z = np.arange(nz)[:, None, None]
    v = (np.sin(math.pi * k[0] * (x + 1) / (nx + 1)) * np.sin(math.pi * k[1] * (y + 1) / (ny + 1))
         * np.sin(math.pi * k[2] * (z + 1) / (nz + 1)))
    lam = sum(2.0 * math.cos(math.pi * kd / (nd + 1)) - 2.0 for kd, nd in zip(k, shape))
    return v, lam


@pytest.mark.parametrize("k", [(2, 3, 1), (11, 1, 8), (5, 9, 4)])
def test_discrete_eigenmode_3d_closed_form(k):
    """A Dirichlet eigenmode v of the 7-point operator (L v = lam v) evolves under
    eq.(3) as phi^n = v cos(n theta), cos(theta) = 1 + C^2 lam / 2, exactly in
    exact arithmetic.  Unequal grid edges catch transposed axes."""
    shape = (12, 10, 9)
    v, lam = _mode(shape, k)
    c2 = 0.25                                   # c = 1, dt = 0.5, dx = 1
    theta = math.acos(1.0 + c2 * lam / 2.0)
    c = np.ones(v.shape)
    steps = 200
    phi, prev, _ = oracle.dense_run(c, 0.5, 1.0, steps, np.float64, phi=v,
                                    phi_prev=v * math.cos(theta))
    assert np.max(np.abs(phi - v * math.cos(steps * theta))) < 1e-11
    assert np.max(np.abs(prev - v * math.cos((steps - 1) * theta))) < 1e-11
    phi32, _, _ = oracle.dense_run(c.astype(np.float32), 0.5, 1.0, steps, np.float32,
                                   phi=v, phi_prev=v * math.cos(theta))
    assert np.max(np.abs(phi32 - v * math.cos(steps * theta))) < 2e-4


def test_energy_conserved_heterogeneous_media():
    """With D = diag(C^2) > 0 and A = -L symmetric, eq.(3) conserves
    E = |phi^{n+1} - phi^n|^2_{D^-1} + <phi^{n+1}, A phi^n> (no sources)."""
    rng = np.random.default_rng(11)
    nz, ny, nx = 13, 15, 17
    c = rng.uniform(0.5, 1.0, (nz, ny, nx))
    dt = 0.55                                    # max Courant 0.55 < 1/sqrt(3)
    D = (c * dt) ** 2
    phi = rng.standard_normal((nz, ny, nx))
    prev = rng.standard_normal((nz, ny, nx))
    energies = []
    for _ in range(240):
        new, cur, _ = oracle.dense_run(c, dt, 1.0, 1, np.float64, phi=phi, phi_prev=prev)
        energies.append(np.sum((new - cur) ** 2 / D) - np.sum(new * _laplacian(cur)))
        phi, prev = new, cur
    e = np.array(energies)
    assert e[0] > 0
    assert np.max(np.abs(e - e[0])) / e[0] < 1e-12


def test_energy_detects_wrong_operator():
    """Sanity of the pin itself: the same energy is NOT conserved for a field
    advanced with a Laplacian that is missing the z-neighbours."""
    rng = np.random.default_rng(3)
    u = rng.standard_normal((7, 8, 9))
    um = rng.standard_normal((7, 8, 9))
    D = 0.2

    def bad_step(u, um):
        p = np.pad(u, 1)
        lap = (p[1:-1, 1:-1, 2:] + p[1:-1, 1:-1, :-2] + p[1:-1, 2:, 1:-1] + p[1:-1, :-2, 1:-1]
               - 6.0 * u)
        return 2 * u - um + D * lap, u

    es = []
    for _ in range(50):
        un, uc = bad_step(u, um)
        es.append(np.sum((un - uc) ** 2 / D) - np.sum(un * _laplacian(uc)))
        u, um = un, uc
    assert np.max(np.abs(np.array(es) - es[0])) / abs(es[0]) > 1e-3


def test_cfl_closed_form_eq4():
    r = 1.0 / math.sqrt(3.0)
    assert oracle.cfl_ok(1.0, r, 1.0)
    assert oracle.cfl_ok(3000.0, 0.5 / 3000.0, 1.0)
    assert not oracle.cfl_ok(1.0, r * 1.0001, 1.0)
    assert oracle.cfl_ok(1.0, 1.0, 1.0, ndim=1)
    assert not oracle.cfl_ok(1.0, 1.0, 1.0, ndim=3)
    assert oracle.cfl_ok(2.0, r / 2.0 * 2.0, 2.0)        # depends on c dt / dx only


def test_cfl_blowup_above_and_bounded_below():
    """Above the limit of eq.(4) the highest mode grows geometrically; just
    below it every mode stays bounded."""
    rng = np.random.default_rng(5)
    shape = (16, 16, 16)
    phi0 = rng.standard_normal(shape)
    c = np.ones(shape)
    r = 1.0 / math.sqrt(3.0)
    hi, _, _ = oracle.dense_run(c, r * 1.02, 1.0, 400, np.float64, phi=phi0, phi_prev=phi0)
    lo, _, _ = oracle.dense_run(c, r * 0.999, 1.0, 400, np.float64, phi=phi0, phi_prev=phi0)
    assert np.max(np.abs(hi)) > 1e6 * np.max(np.abs(phi0))
    assert np.max(np.abs(lo)) < 50 * np.max(np.abs(phi0))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_point_source_symmetry_bitexact(dtype):
    """Odd grid, centred source, homogeneous media: the x, y, z mirrors and the
    x<->y swap are exact with the pairwise neighbour sum; x<->z within rounding."""
    n = 33
    c = np.ones((n, n, n))
    w = np.sin(np.linspace(0, 3, 40)) * np.exp(-np.linspace(0, 3, 40))
    phi, _, _ = oracle.dense_run(c, 0.5, 1.0, 60, dtype, sources=[((16, 16, 16), w)])
    assert values_equal(phi, phi[:, :, ::-1])
    assert values_equal(phi, phi[:, ::-1, :])
    assert values_equal(phi, phi[::-1, :, :])
    assert values_equal(phi, phi.transpose(0, 2, 1))
    tol = 1e-5 if dtype == np.float32 else 1e-13
    assert np.max(np.abs(phi - phi.transpose(2, 1, 0))) <= tol * np.max(np.abs(phi))


def test_reciprocity_heterogeneous():
    """For u^{n+1} = 2u^n - u^{n-1} + D L u^n + f^n e_s with symmetric L:
    C2_s * trace(s -> r) == C2_r * trace(r -> s)."""
    rng = np.random.default_rng(21)
    nz, ny, nx = 10, 11, 12
    c = rng.uniform(0.6, 1.0, (nz, ny, nx))
    dt = 0.5
    s, r = (2, 3, 4), (9, 7, 6)
    w = rng.standard_normal(25)
    _, _, t_sr = oracle.dense_run(c, dt, 1.0, 80, np.float64, sources=[(s, w)], receivers=[r])
    _, _, t_rs = oracle.dense_run(c, dt, 1.0, 80, np.float64, sources=[(r, w)], receivers=[s])
    Ds = (c[s[2], s[1], s[0]] * dt) ** 2
    Dr = (c[r[2], r[1], r[0]] * dt) ** 2
    a, b = Ds * t_sr[:, 0], Dr * t_rs[:, 0]
    assert np.max(np.abs(a)) > 1e-6
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(a))
    assert np.max(np.abs(t_sr[:, 0] - t_rs[:, 0])) > 1e-6 * np.max(np.abs(t_sr))   # media matter


def test_source_sample_timing_and_start_step():
    """Sample k of a source started at step t0 enters phi^{t0+k+1} additively."""
    c = np.ones((5, 5, 5))
    w = np.array([1.0, 2.0, 3.0])
    phi, _, tr = oracle.dense_run(c, 0.5, 1.0, 1, np.float64, sources=[((2, 2, 2), w)],
                                  receivers=[(2, 2, 2)])
    assert phi[2, 2, 2] == 1.0 and np.count_nonzero(phi) == 1 and tr[0, 0] == 1.0
    # delayed start: nothing before step 4, then samples in order
    _, _, tr = oracle.dense_run(c, 0.0, 1.0, 8, np.float64, sources=[((2, 2, 2), w, 4)],
                                receivers=[(2, 2, 2)])
    # with C^2 = 0, phi^{n+1} = 2 phi^n - phi^{n-1} + w: second sum of the samples
    seq = np.zeros(8)
    u, um = 0.0, 0.0
    for n in range(8):
        un = 2 * u - um + (w[n - 4] if 4 <= n < 7 else 0.0)
        seq[n] = un
        u, um = un, u
    assert np.array_equal(tr[:, 0], seq)


def test_paper_closed_forms():
    """eq.(5) with the paper's scenario values (c = 340 m/s, dt = 1e-3 s,
    dx = 1 m) and 20-node cells gives 29.4 -> an update every 29 steps, as in
    the Results section; the 2000^3 speed-up 70 s * 8 / 43 s = 13.0; the
    memory factor 1 / 0.0407 = 24.6 ~ 25; eq.(6) A = alpha^n."""
    n = oracle.update_interval(1.0, 20.0, 340.0, 1e-3)
    assert abs(n - 29.41176470588235) < 1e-12 and int(n) == 29
    assert round(70.0 * 8.0 / 43.0) == 13
    assert round(1.0 / 0.0407) == 25
    assert oracle.decay_total(0.5, 3) == 0.125
    assert abs(oracle.decay_total(0.1 ** 0.1, 20) - 0.01) < 1e-15
