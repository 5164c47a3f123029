"""The HBM ceiling probe that the stencil's roofline fraction is compared
with: it must compute its sums and report a bandwidth below the HBM peak."""
import pytest

pytestmark = pytest.mark.gpu
tcm = pytest.importorskip("paper_1702_00216_amd")


@pytest.mark.parametrize("nread", [1, 2, 3])
def test_hbm_probe_sums_and_bandwidth(nread):
    print(f"\n[case] hbm probe nread={nread}", flush=True)
    r = tcm.hbm_probe(nread, n=1 << 26, wg_per_cu=8, reps=3)
    assert r["result_ok"]
    assert r["bytes"] == (nread + 1) * 4 * (1 << 26)
    # 8 TB/s is the published peak; anything near or above it is a timing bug
    assert 500.0 < r["GBps"] < 8000.0
