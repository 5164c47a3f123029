"""Write the stored expected values of the full-size workloads.

Calls only the CPU oracle (oracle/) and the input generators (tcm_inputs/).
Usage:  python tests/golden/make_golden.py c2 [--sweep]
        python tests/golden/make_golden.py c5
        python tests/golden/make_golden.py c4
        python tests/golden/make_golden.py c4tau      (after c4)
        python tests/golden/make_golden.py c2k8
        python tests/golden/make_golden.py c5resid

c2: the 512^3 two-layer workload, 2000 steps.  Stores
  * the relative L2 error at the last step against the FP64 dense oracle of
    the FP32 dense oracle and of the FP32 CPU TCM at the workload's
    thresholds (trigger 1e-6, retire 1e-7 of the source peak), and with
    --sweep at trigger = k * peak (retire = trigger / 10) for k in
    {1e-10, 1e-9, 1e-8, 1e-7, 1e-6, 1e-5};
  * SHA-256 of the CPU TCM's final phi^n and phi^{n-1} (float32, -0 -> +0),
    values at 4096 seeded sample nodes, traces at 8 receivers, and its
    statistics (peak active cells, activations, retirements, node updates).
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import tcm_inputs as ti  # noqa: E402


def digest(a: np.ndarray) -> str:
    a = np.ascontiguousarray(a, dtype=np.float32) + np.float32(0.0)   # -0 -> +0
    return hashlib.sha256(a.tobytes()).hexdigest()


def relerr(a, ref) -> float:
    return float(np.linalg.norm(a.astype(np.float64) - ref) / np.linalg.norm(ref))


def c2_receivers(shape):
    nx, ny, nz = shape
    return [(nx // 2, ny // 2, nz // 4), (nx // 4, ny // 2, nz // 8), (nx - 3, 5, 2),
            (nx // 2, ny // 2, nz - 2), (17, ny - 9, nz // 2), (nx // 2 + 1, ny // 2, nz // 2),
            (3, 3, 3), (nx // 3, 2 * ny // 3, 3 * nz // 5)]


def sample_nodes(shape, n=4096, seed=77):
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    return np.stack([rng.integers(0, nx, n), rng.integers(0, ny, n), rng.integers(0, nz, n)], 1)


def log(m):
    print(f"[golden {time.strftime('%H:%M:%S')}] {m}", flush=True)


def make_c2(sweep: bool):
    w = ti.c2()
    c = w.layered.dense(*w.shape)
    out_path = os.path.join(HERE, "c2_golden.json")
    res = json.load(open(out_path)) if os.path.exists(out_path) else {}
    res["workload"] = {"shape": w.shape, "steps": w.steps, "dt": w.dt, "source": w.source,
                       "trigger": w.trigger, "retire": w.retire, "peak": w.wavelet.peak}
    t0 = time.time()
    ref, _, _ = oracle.dense_run(c.astype(np.float64), w.dt, w.dx, w.steps, np.float64,
                                 sources=[(w.source, w.wavelet.w32.astype(np.float64))])
    log(f"FP64 dense done in {time.time() - t0:.0f} s")
    t0 = time.time()
    d32, _, _ = oracle.dense_run(c, w.dt, w.dx, w.steps, np.float32, sources=[(w.source, w.wavelet.w32)])
    res["err_dense_fp32"] = relerr(d32, ref)
    res["dense_fp32_sha256"] = digest(d32)
    del d32
    log(f"FP32 dense done in {time.time() - t0:.0f} s, err {res['err_dense_fp32']:.3e}")
    rec = c2_receivers(w.shape)
    t0 = time.time()
    t = oracle.TCM(c, w.dt, w.dx, np.float32(w.trigger), np.float32(w.retire))
    t.add_source(w.source, w.wavelet.w32)
    t.set_receivers(rec)
    rc, tr = t.step(w.steps, traces=True)
    assert rc == 0
    phi, prev = t.read(0), t.read(1)
    st = t.stats()
    t.close()
    log(f"FP32 CPU TCM done in {time.time() - t0:.0f} s")
    nodes = sample_nodes(w.shape)
    res["tcm"] = {"err": relerr(phi, ref), "phi_sha256": digest(phi), "prev_sha256": digest(prev),
                  "stats": st, "receivers": rec, "traces_sha256": digest(tr),
                  "traces_last": tr[-1].tolist(),
                  "sample_nodes": nodes.tolist(),
                  "sample_phi": phi[nodes[:, 2], nodes[:, 1], nodes[:, 0]].tolist()}
    json.dump(res, open(out_path, "w"))
    log(f"TCM err {res['tcm']['err']:.3e}, stats {st}")
    if sweep:
        res.setdefault("sweep", {})
        for k in (1e-10, 1e-9, 1e-8, 1e-7, 1e-6, 1e-5):
            t0 = time.time()
            trig = np.float32(k * w.wavelet.peak)
            t = oracle.TCM(c, w.dt, w.dx, trig, np.float32(trig / 10))
            t.add_source(w.source, w.wavelet.w32)
            assert t.step(w.steps) == 0
            p = t.read(0)
            s = t.stats()
            t.close()
            res["sweep"][f"{k:g}"] = {"err": relerr(p, ref), "updates": s["updates"],
                                      "peak_active": s["peak_active"], "sha256": digest(p)}
            json.dump(res, open(out_path, "w"))
            log(f"sweep {k:g}: err {res['sweep'][f'{k:g}']['err']:.3e} updates {s['updates']:.3e} "
                f"({time.time() - t0:.0f} s)")


def make_c5():
    """256^3 lognormal model, 1000 steps, 128 receivers on z = 240, misfit
    against FP64 traces of the +2 % anomaly model.  Stores the FP64 adjoint
    gradient (O3) on every 8th node per axis, at 4096 seeded nodes, and at 32
    nodes (seed 55, |grad| > 1e-3 max) together with FP64 central differences
    of J (h = 1e-4 c) there."""
    w = ti.c5()
    shape = w.shape
    c = ti.lattice_to_dense(w.lattice, shape).astype(np.float64)
    c_true = ti.lattice_to_dense(ti.c5_true_lattice(w.lattice), shape).astype(np.float64)
    src = [(w.source, w.wavelet.w32.astype(np.float64))]
    rec = w.receivers
    nt = w.steps
    t0 = time.time()
    d_obs = oracle.dense_run(c_true, w.dt, w.dx, nt, np.float64, sources=src, receivers=rec)[2]
    tr = oracle.dense_run(c, w.dt, w.dx, nt, np.float64, sources=src, receivers=rec)[2]
    resid = tr - d_obs
    J0 = 0.5 * float(np.sum(resid ** 2))
    log(f"c5 forward runs done in {time.time() - t0:.0f} s, J = {J0:.6e}")
    t0 = time.time()
    g = oracle.adjoint_f64(c, w.dt, w.dx, src, rec, resid, ckpt=50)
    log(f"c5 FP64 adjoint done in {time.time() - t0:.0f} s")
    gmax = float(np.max(np.abs(g)))
    rng = np.random.default_rng(55)
    cand = np.argwhere(np.abs(g) > 1e-3 * gmax)
    pick = cand[rng.choice(len(cand), size=32, replace=False)]
    res = {"workload": {"shape": shape, "steps": nt, "dt": w.dt, "source": w.source,
                        "receivers": rec.tolist()},
           "J": J0, "grad_norm": float(np.linalg.norm(g)), "grad_max": gmax,
           "sub8": {"step": 8, "file": "c5_grad_sub8.npy"}}
    np.save(os.path.join(HERE, "c5_grad_sub8.npy"), g[::8, ::8, ::8].astype(np.float32))
    nodes = sample_nodes(shape, seed=78)
    res["sample_nodes"] = nodes.tolist()
    res["sample_grad"] = g[nodes[:, 2], nodes[:, 1], nodes[:, 0]].tolist()
    fd_cells = []
    for (z, y, x) in pick:
        h = 1e-4 * c[z, y, x]
        cp = c.copy()
        cp[z, y, x] += h
        Jp = 0.5 * float(np.sum((oracle.dense_run(cp, w.dt, w.dx, nt, np.float64, sources=src,
                                                  receivers=rec)[2] - d_obs) ** 2))
        cp[z, y, x] -= 2 * h
        Jm = 0.5 * float(np.sum((oracle.dense_run(cp, w.dt, w.dx, nt, np.float64, sources=src,
                                                  receivers=rec)[2] - d_obs) ** 2))
        fd = (Jp - Jm) / (2 * h)
        fd_cells.append({"xyz": [int(x), int(y), int(z)], "fd": fd, "adjoint": float(g[z, y, x])})
        res["fd_cells"] = fd_cells
        json.dump(res, open(os.path.join(HERE, "c5_golden.json"), "w"))
        log(f"fd ({x},{y},{z}): fd {fd:.6e} adjoint {g[z, y, x]:.6e}")


def make_c5resid():
    """The residual (FP64 traces of the model minus FP64 traces of the +2 %
    anomaly model) that the stored c5 adjoint gradient was computed with,
    rounded to FP32 (c5_resid.npy), so the GPU adjoint can be fed the same
    input."""
    w = ti.c5()
    c = ti.lattice_to_dense(w.lattice, w.shape).astype(np.float64)
    c_true = ti.lattice_to_dense(ti.c5_true_lattice(w.lattice), w.shape).astype(np.float64)
    src = [(w.source, w.wavelet.w32.astype(np.float64))]
    d_obs = oracle.dense_run(c_true, w.dt, w.dx, w.steps, np.float64, sources=src, receivers=w.receivers)[2]
    tr = oracle.dense_run(c, w.dt, w.dx, w.steps, np.float64, sources=src, receivers=w.receivers)[2]
    resid = tr - d_obs
    J = 0.5 * float(np.sum(resid ** 2))
    g = json.load(open(os.path.join(HERE, "c5_golden.json")))
    assert abs(J - g["J"]) <= 1e-12 * abs(g["J"]), (J, g["J"])
    np.save(os.path.join(HERE, "c5_resid.npy"), resid.astype(np.float32))
    log(f"c5 resid saved, J = {J:.6e}")


def make_c2k8():
    """The 512^3 two-layer workload with the activation update every 8 steps
    (eq.(5) with 8-node cells at Courant 0.5) and the 26-cell lookahead:
    error against FP64 dense, final-field hashes and statistics of the CPU TCM,
    at the workload thresholds and at trigger 1e-9 / retire 1e-10 of the peak."""
    w = ti.c2()
    c = w.layered.dense(*w.shape)
    out_path = os.path.join(HERE, "c2k8_golden.json")
    res = {"interval": 8, "workload": {"shape": w.shape, "steps": w.steps}}
    t0 = time.time()
    ref, _, _ = oracle.dense_run(c.astype(np.float64), w.dt, w.dx, w.steps, np.float64,
                                 sources=[(w.source, w.wavelet.w32.astype(np.float64))])
    log(f"FP64 dense done in {time.time() - t0:.0f} s")
    for name, trig, ret in (("workload", w.trigger, w.retire),
                            ("1e-09", 1e-9 * w.wavelet.peak, 1e-10 * w.wavelet.peak)):
        t0 = time.time()
        t = oracle.TCM(c, w.dt, w.dx, np.float32(trig), np.float32(ret), interval=8)
        t.add_source(w.source, w.wavelet.w32)
        assert t.step(w.steps) == 0
        phi, prev = t.read(0), t.read(1)
        st = t.stats()
        t.close()
        res[name] = {"trigger": float(np.float32(trig)), "retire": float(np.float32(ret)),
                     "err": relerr(phi, ref), "phi_sha256": digest(phi), "prev_sha256": digest(prev),
                     "stats": st}
        json.dump(res, open(out_path, "w"))
        log(f"c2k8 {name}: err {res[name]['err']:.3e} updates {st['updates']:.3e} ({time.time() - t0:.0f} s)")


C4_TAU_SHOTS = (17, 61, 41)      # the three smallest shots (about 3e6 nodes each)


def make_c4tau():
    """Shots 17, 61 and 41 of the 64-shot workload at its thresholds (trigger
    1e-6 / retire 1e-7 of the source peak), 1500 steps: SHA-256 of the FP32
    CPU TCM's final phi^n and phi^{n-1}, and its statistics."""
    path = os.path.join(HERE, "c4_golden.json")
    res = json.load(open(path))
    shots = ti.c4_shots()
    res["tau_shots"] = []
    for i in C4_TAU_SHOTS:
        s = shots[i]
        t0 = time.time()
        t = oracle.TCM(ti.lattice_to_dense(s.lattice, s.shape), s.dt, s.dx, np.float32(s.trigger),
                       np.float32(s.retire))
        t.add_source(s.source, s.wavelet.w32)
        assert t.step(s.steps) == 0
        res["tau_shots"].append({"shot": i, "shape": s.shape, "trigger": float(np.float32(s.trigger)),
                                 "retire": float(np.float32(s.retire)),
                                 "phi_sha256": digest(t.read(0)), "prev_sha256": digest(t.read(1)),
                                 "stats": t.stats()})
        t.close()
        json.dump(res, open(path, "w"))
        log(f"{s.name} {s.shape} at the workload thresholds: {time.time() - t0:.0f} s")


def make_c4():
    """Shots 0-3 of the 64-shot workload at threshold 0: SHA-256 of the FP32
    dense oracle's final phi^n (equal to the TCM at threshold 0)."""
    shots = ti.c4_shots()[:4]
    res = {"shots": []}
    for s in shots:
        t0 = time.time()
        cd = ti.lattice_to_dense(s.lattice, s.shape)
        phi, _, _ = oracle.dense_run(cd, s.dt, s.dx, s.steps, np.float32,
                                     sources=[(s.source, s.wavelet.w32)])
        res["shots"].append({"shape": s.shape, "source": s.source, "phi_sha256": digest(phi)})
        json.dump(res, open(os.path.join(HERE, "c4_golden.json"), "w"))
        log(f"{s.name} {s.shape}: {time.time() - t0:.0f} s")


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "c2"
    if which == "c2":
        make_c2("--sweep" in sys.argv)
    elif which == "c5":
        make_c5()
    elif which == "c4":
        make_c4()
    elif which == "c4tau":
        make_c4tau()
    elif which == "c2k8":
        make_c2k8()
    elif which == "c5resid":
        make_c5resid()
    else:
        raise SystemExit(f"unknown workload {which}")
