"""bench.py helpers that decide what the JSON line reports: the launch shape
of the stencil and the HBM traffic read from the committed counter
summaries, which may only be used for the kernel source and launch shape
they were taken on."""
import glob
import os
import types

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_launch_shape_names_tuned_given_and_default_shapes():
    args = types.SimpleNamespace(blocks_per_wg=0, blocks_per_wave=0, wg_per_cu=0)
    assert bench.launch_shape(None, args) == "4x1@3"           # the library's default
    args = types.SimpleNamespace(blocks_per_wg=8, blocks_per_wave=2, wg_per_cu=0)
    assert bench.launch_shape(None, args) == "8x2@3"
    args = types.SimpleNamespace(blocks_per_wg=8, blocks_per_wave=1, wg_per_cu=2)
    assert bench.launch_shape(None, args) == "8x1@2"
    tuned = {"blocks_per_wg": 2, "blocks_per_wave": 1, "wg_per_cu": 8}
    assert bench.launch_shape(tuned, args) == "2x1@8"


def test_kernel_source_hash_covers_the_whole_function():
    h = bench.kernel_source_hash("k_block_step")
    g = bench.kernel_source_hash("k_plan")
    assert len(h) == 16 and len(g) == 16 and h != g


def test_traffic_summaries_are_complete_and_keyed():
    files = glob.glob(os.path.join(ROOT, "profiles", "*_traffic.md"))
    assert files
    for p in files:
        kernel, workload = os.path.basename(p)[:-len("_traffic.md")].rsplit("_", 1)
        kv = dict(line.strip().split("=", 1) for line in open(p) if "=" in line and not line.startswith(" "))
        assert f"{kernel}_source_sha256_16" in kv and int(kv["traffic_bytes_per_dispatch"]) > 0
        assert int(kv["dispatch_mean_algorithmic_bytes"]) > 0
        t = bench.measured_traffic(kernel, workload, kv.get("launch_shape"))
        if kv[f"{kernel}_source_sha256_16"] == bench.kernel_source_hash(kernel):
            assert t == int(kv["traffic_bytes_per_dispatch"])
        else:
            assert t is None                                   # taken on other code: not reported
        if "launch_shape" in kv:
            assert bench.measured_traffic(kernel, workload, "2x2@99") is None
