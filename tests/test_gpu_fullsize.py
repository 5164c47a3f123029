"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times (per-launch event timing, default grid), against values written by
tests/golden/make_golden.py from the CPU oracle, or against the oracle on a
crop where the stencil's light cone makes the crop exact."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
import tcm_inputs as ti
from conftest import values_equal

pytestmark = pytest.mark.gpu
tcm = pytest.importorskip("paper_1702_00216_amd")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def announce(msg):
    print(f"\n[case] {msg}", flush=True)


def digest(a):
    a = np.ascontiguousarray(a, dtype=np.float32) + np.float32(0.0)
    return hashlib.sha256(a.tobytes()).hexdigest()


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_c2_full_run_bitexact_to_cpu_tcm():
    """512^3 two-layer, 2000 steps, trigger 1e-6 / retire 1e-7: the whole final
    field (both levels), the traces and the work statistics equal the CPU TCM."""
    announce("C2 full size vs stored CPU TCM result")
    g = load("c2_golden.json")["tcm"]
    w = ti.c2()
    sim = tcm.Simulation(w.shape, w.dx, w.dt, w.layered, w.trigger, w.retire, timing=True)
    sim.add_source(w.source, w.wavelet.w32)
    sim.set_receivers(g["receivers"])
    sim.step(w.steps)
    st = sim.stats()
    o = g["stats"]
    assert st["step"] == o["step"] and st["active_blocks"] == o["active"]
    assert st["peak_active_blocks"] == o["peak_active"]
    assert st["activations"] == o["activations"] and st["retirements"] == o["retirements"]
    assert st["cell_updates"] == o["updates"]
    phi = sim.read(0)
    nodes = np.array(g["sample_nodes"])
    assert values_equal(phi[nodes[:, 2], nodes[:, 1], nodes[:, 0]], np.array(g["sample_phi"], np.float32))
    assert digest(phi) == g["phi_sha256"]
    del phi
    assert digest(sim.read(1)) == g["prev_sha256"]
    tr = sim.read_traces()
    assert values_equal(tr[-1], np.array(g["traces_last"], np.float32))
    assert digest(tr) == g["traces_sha256"]


def test_c2_equal_error_run_bitexact_to_cpu_tcm():
    """The run the equal-error speed-up is quoted on: 512^3 two-layer, 2000
    steps, trigger 1e-9 / retire 1e-10 of the source peak, activation update
    every step.  The final field and the work equal the CPU TCM's (threshold
    sweep of c2_golden.json)."""
    announce("C2 trigger 1e-9 / retire 1e-10 vs stored CPU TCM result")
    g = load("c2_golden.json")["sweep"]["1e-09"]
    w = ti.c2()
    trig = np.float32(1e-9 * w.wavelet.peak)
    ret = np.float32(trig / 10)
    sim = tcm.Simulation(w.shape, w.dx, w.dt, w.layered, float(trig), float(ret), timing=True)
    sim.add_source(w.source, w.wavelet.w32)
    sim.step(w.steps)
    st = sim.stats()
    assert st["step"] == w.steps and st["error"] == 0
    assert st["cell_updates"] == g["updates"] and st["peak_active_blocks"] == g["peak_active"]
    assert digest(sim.read(0)) == g["sha256"]


@pytest.mark.parametrize("name", ["workload", "1e-09"])
def test_c2_interval8_full_run_bitexact_to_cpu_tcm(name):
    """512^3 two-layer, 2000 steps with the activation update every 8 steps
    (eq.(5)) and the 26-neighbour lookahead, at the workload thresholds and at
    trigger 1e-9 / retire 1e-10 of the peak: both final levels and the work
    statistics equal the CPU TCM."""
    announce(f"C2 interval 8 ({name}) vs stored CPU TCM result")
    g = load("c2k8_golden.json")
    o = g[name]
    w = ti.c2()
    sim = tcm.Simulation(w.shape, w.dx, w.dt, w.layered, o["trigger"], o["retire"], timing=True,
                         trigger_interval=g["interval"])
    sim.add_source(w.source, w.wavelet.w32)
    sim.step(w.steps)
    st = sim.stats()
    s = o["stats"]
    assert st["step"] == s["step"] and st["active_blocks"] == s["active"]
    assert st["peak_active_blocks"] == s["peak_active"]
    assert st["activations"] == s["activations"] and st["retirements"] == s["retirements"]
    assert st["cell_updates"] == s["updates"]
    assert digest(sim.read(0)) == o["phi_sha256"]
    assert digest(sim.read(1)) == o["prev_sha256"]


def test_c3_virtual_4096_first_steps_match_cpu_tcm_on_crop():
    """Virtual 4096^3 domain with the 64 GB pool cap: after 200 steps every
    nonzero node lies within 200 nodes of the source, so the CPU TCM on the
    512^3 crop around it computes the same field bit for bit."""
    announce("C3 4096^3 first 200 steps vs CPU TCM on a 512^3 crop")
    w = ti.c3()
    steps, edge = 200, 512
    sim = tcm.Simulation(w.shape, w.dx, w.dt, w.lattice, w.trigger, w.retire,
                         pool_bytes=w.pool_bytes, timing=True)
    sim.add_source(w.source, w.wavelet.w32)
    sim.step(steps)
    o = tuple(s - edge // 2 for s in w.source)
    gpu = sim.read(0, box=(o, (edge,) * 3))
    st = sim.stats()
    assert st["pool_bytes"] <= w.pool_bytes and st["error"] == 0
    c = ti.lattice_to_dense(w.lattice, w.shape, origin=o, extent=(edge,) * 3)
    t = oracle.TCM(c, w.dt, w.dx, np.float32(w.trigger), np.float32(w.retire))
    t.add_source((edge // 2,) * 3, w.wavelet.w32)
    assert t.step(steps) == 0
    assert values_equal(gpu, t.read(0))
    ts = t.stats()
    assert st["active_blocks"] == ts["active"] and st["cell_updates"] == ts["updates"]
    assert st["activations"] == ts["activations"] and st["retirements"] == ts["retirements"]


def test_c4_full_batch_equals_single_shots():
    """64 shots (edges 96..384) over one shared pool, 1500 steps at the
    workload thresholds: shots 17, 61 and 41 equal the CPU TCM (stored
    hashes), and every shot equals its own single-shot run."""
    announce("C4 64-shot batch vs single shots")
    shots = ti.c4_shots()
    b = tcm.Simulation([s.shape for s in shots], 1.0, shots[0].dt, [s.lattice for s in shots],
                       shots[0].trigger, shots[0].retire)
    for i, s in enumerate(shots):
        b.add_source(s.source, s.wavelet.w32, shot=i)
    b.step(shots[0].steps)
    # three shots against the CPU TCM at these thresholds
    for o in load("c4_golden.json")["tau_shots"]:
        i = o["shot"]
        assert np.float32(shots[i].trigger) == np.float32(o["trigger"])
        assert digest(b.read(0, shot=i)) == o["phi_sha256"], i
        assert digest(b.read(1, shot=i)) == o["prev_sha256"], i
    tot = 0
    for i, s in enumerate(shots):
        one = tcm.Simulation(s.shape, 1.0, s.dt, s.lattice, s.trigger, s.retire)
        one.add_source(s.source, s.wavelet.w32)
        one.step(s.steps)
        assert values_equal(b.read(0, shot=i), one.read(0)), i
        tot += one.stats()["cell_updates"]
        one.close()
    assert b.stats()["cell_updates"] == tot


def test_c4_shots_at_threshold_zero_equal_dense_oracle():
    """Shots 0-3 of the batch at threshold 0 equal the FP32 dense oracle."""
    announce("C4 shots 0-3 tau=0 vs stored dense oracle hashes")
    g = load("c4_golden.json")
    shots = ti.c4_shots()[:4]
    b = tcm.Simulation([s.shape for s in shots], 1.0, shots[0].dt, [s.lattice for s in shots], 0.0, 0.0)
    for i, s in enumerate(shots):
        b.add_source(s.source, s.wavelet.w32, shot=i)
    b.step(shots[0].steps)
    for i in range(4):
        assert digest(b.read(0, shot=i)) == g["shots"][i]["phi_sha256"], i


def test_c5_gradient_against_fp64_adjoint_and_finite_differences():
    """256^3, 1000 steps, 128 receivers, checkpoints every 50.
    (1) Parity: fed the oracle's residual, the GPU FP32 gradient matches the
        FP64 adjoint within rel. L2 1e-3 on every 8th node (which includes the
        source and all receiver nodes) and on 4096 seeded nodes.
    (2) End to end: with its own FP32 residual, the GPU gradient matches FP64
        central differences of J at 32 nodes within 1e-2."""
    announce("C5 adjoint vs stored FP64 adjoint and finite differences")
    g = load("c5_golden.json")
    w = ti.c5()
    c = ti.lattice_to_dense(w.lattice, w.shape)
    sim = tcm.Simulation(w.shape, w.dx, w.dt, c, checkpoint_every=50, timing=True)
    sim.add_source(w.source, w.wavelet.w32)
    sim.set_receivers(w.receivers)
    sim.step(w.steps)
    resid_o = np.load(os.path.join(GOLDEN, "c5_resid.npy"))
    grad = sim.adjoint(resid_o)
    # the lattice media themselves (C2 from lattice records in the stencil)
    # give the same gradient bit for bit
    lsim = tcm.Simulation(w.shape, w.dx, w.dt, w.lattice, checkpoint_every=50)
    lsim.add_source(w.source, w.wavelet.w32)
    lsim.set_receivers(w.receivers)
    lsim.step(w.steps)
    assert lsim.stats()["lattice_cell_updates"] > 0
    assert np.array_equal(lsim.adjoint(resid_o), grad)
    lsim.close()
    sub = np.load(os.path.join(GOLDEN, g["sub8"]["file"])).astype(np.float64)
    e_sub = np.linalg.norm(grad[::8, ::8, ::8] - sub) / np.linalg.norm(sub)
    nodes = np.array(g["sample_nodes"])
    ref = np.array(g["sample_grad"])
    e_smp = np.linalg.norm(grad[nodes[:, 2], nodes[:, 1], nodes[:, 0]] - ref) / np.linalg.norm(ref)
    # end to end: observed data from the GPU forward of the anomaly model
    c_true = ti.lattice_to_dense(ti.c5_true_lattice(w.lattice), w.shape)
    obs = tcm.Simulation(w.shape, w.dx, w.dt, c_true)
    obs.add_source(w.source, w.wavelet.w32)
    obs.set_receivers(w.receivers)
    obs.step(w.steps)
    d_obs = obs.read_traces().astype(np.float64)
    obs.close()
    resid = (sim.read_traces().astype(np.float64) - d_obs).astype(np.float32)
    grad_e2e = sim.adjoint(resid)
    fd_err = [abs(grad_e2e[z, y, x] - f["fd"]) / abs(f["fd"])
              for f in g["fd_cells"] for (x, y, z) in [f["xyz"]]]
    e2e_sub = np.linalg.norm(grad_e2e[::8, ::8, ::8] - sub) / np.linalg.norm(sub)
    # the residual is the trace difference of a 2 % model change: the FP32
    # forward's rounding of the traces is a much larger part of it than of the
    # traces, and the gradient is linear in the residual
    e_res = float(np.linalg.norm(resid.astype(np.float64) - resid_o) / np.linalg.norm(resid_o))
    print(f"C5 same residual: rel-L2 vs FP64 adjoint (every 8th node) {e_sub:.3e}, (4096 nodes) "
          f"{e_smp:.3e}; end to end: max rel err vs FD over {len(fd_err)} nodes {max(fd_err):.3e}, "
          f"rel-L2 every 8th node {e2e_sub:.3e} (FP32 residual vs FP64: {e_res:.3e})")
    assert len(fd_err) == 32
    assert e_sub <= 1e-3 and e_smp <= 1e-3 and max(fd_err) <= 1e-2
    assert e2e_sub <= 5e-3
