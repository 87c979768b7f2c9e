"""Host logic of bench.py (no GPU): the one-GPU guard, the roofline arithmetic
of the dominant kernel, the committed counter figures and their source digest,
and the Jacobi sweep count of the Euclidean variant."""
import json
import math
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def _kt(**over):
    k = lambda ms, launches, voxels: dict(ms=ms, launches=launches, voxels=voxels)  # noqa: E731
    kt = {"predict": k(50.0, 100, 3.0e10), "compare": k(80.0, 100, 3.0e10),
          "reinit": k(100.0, 100, 3.0e10), "reinit_sweep": k(0.0, 0, 0), "plan": k(5.0, 700, 0)}
    kt.update(over)
    return kt


def test_roofline_of_the_dominant_kernel():
    r = bench.roofline(_kt(), 4, physics=False)
    assert r["kernel"] == "reinit" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    # two values of 4 bytes per grain voxel over 100 ms
    assert r["achieved"] == pytest.approx(2 * 4 * 3.0e10 / 0.1 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["avg_launch_ms"] == pytest.approx(1.0)
    assert r["alg_bytes_per_launch"] == pytest.approx(2 * 4 * 3.0e10 / 100)
    assert set(r["per_kernel"]) == {"predict", "compare", "reinit"}
    assert r["traffic"] is None


def test_roofline_counts_the_correction_and_the_jacobi_sweeps():
    r = bench.roofline(_kt(), 4, physics=True)
    assert r["kernel"] == "reinit"
    assert r["per_kernel"]["compare"]["GBs"] == pytest.approx((2 * 4 + 4) * 3.0e10 / 0.08 / 1e9, rel=1e-6)
    assert r["per_kernel"]["predict"]["GBs"] == pytest.approx((2 * 4 + 4) * 3.0e10 / 0.05 / 1e9, rel=1e-6)
    r = bench.roofline(_kt(reinit_sweep=dict(ms=400.0, launches=3200, voxels=3.0e10)), 4, physics=False, sweeps=16)
    assert r["kernel"] == "reinit_sweep"
    assert r["achieved"] == pytest.approx(2 * 16 * 4 * 3.0e10 / 0.4 / 1e9)


def test_step_algorithmic_bytes():
    # three sweeps, each reading and writing every grain voxel once
    assert bench.step_alg_bytes(4, False) == 24
    assert bench.step_alg_bytes(8, False) == 48
    # the ID-field: written by the corrector, read by the predictor
    assert bench.step_alg_bytes(4, True) == 32


def test_recorded_traffic_follows_the_sources(monkeypatch, tmp_path):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    (tmp_path / "traffic_compare_w_fp32.md").write_text(
        f"# summary\n- source_sha256: `{bench.source_digest()}`\n- hbm_bytes_per_gv: `8.8`\n")
    assert bench.recorded_traffic("compare", "fp32", "w") == pytest.approx(8.8)
    r = bench.roofline(_kt(compare=dict(ms=300.0, launches=100, voxels=3.0e10)), 4, physics=False,
                       workload="w", precision="fp32")
    assert r["kernel"] == "compare"
    assert r["traffic"] == pytest.approx(8.8 * 3.0e10 / 100)
    assert r["traffic_over_algorithmic"] == pytest.approx(8.8 / 8)
    assert bench.recorded_traffic("compare", "fp32", "no_such_workload") is None
    monkeypatch.setattr(bench, "source_digest", lambda: "0" * 64)
    assert bench.recorded_traffic("compare", "fp32", "w") is None


def test_recorded_error_vs_oracle(monkeypatch, tmp_path):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    assert bench.recorded_error_vs_oracle("fp32") is None
    rec = dict(workload="config 1", steps=20, first_divergence_step=None, band_max_abs=1e-4, per_step=[{}])
    (tmp_path / "error_vs_oracle_fp32.md").write_text(
        f"# summary\n- source_sha256: `{bench.source_digest()}`\n- {json.dumps(rec)}\n")
    r = bench.recorded_error_vs_oracle("fp32")
    assert r["source_match"] and r["workloads"]["config 1"] == dict(steps=20, first_divergence_step=None,
                                                                    band_max_abs=1e-4)
    monkeypatch.setattr(bench, "source_digest", lambda: "0" * 64)
    assert not bench.recorded_error_vs_oracle("fp32")["source_match"]


def test_committed_traffic_summaries_name_their_figures():
    d = os.path.join(ROOT, "profiles")
    for f in (os.listdir(d) if os.path.isdir(d) else []):
        if not f.startswith("traffic_"):
            continue
        text = open(os.path.join(ROOT, "profiles", f)).read()
        assert "source_sha256" in text and "hbm_bytes_per_gv" in text, f


@pytest.mark.parametrize("dim,W", [(2, 6.0), (3, 8.0), (3, 5.5), (2, 16.0)])
def test_euclid_sweep_count(dim, W):
    K = bench.euclid_sweeps(dim, W)
    assert K % 2 == 0 and K >= math.ceil(math.sqrt(dim) * W) + 1 and K <= math.ceil(math.sqrt(dim) * W) + 2
