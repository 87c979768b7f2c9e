"""Host logic of bench.py (no GPU): the one-GPU guard, the roofline arithmetic
of the dominant kernel, the committed counter figures and their source digest,
and the Jacobi sweep count of the Euclidean variant."""
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


def _res(physics=False, sweeps=0):
    k = lambda ms, launches, voxels: dict(ms=ms, launches=launches, voxels=voxels)  # noqa: E731
    return dict(physics=physics, sweeps=sweeps, kernels={
        "conv_xy": k(50.0, 100, 3.0e10), "conv_z": k(0.0, 0, 0), "compare": k(80.0, 100, 3.0e10),
        "reinit_xy": k(100.0, 200, 3.0e10), "reinit_z": k(60.0, 100, 3.0e10),
        "reinit_sweep": k(0.0, 0, 0)})


def test_roofline_of_the_dominant_kernel():
    r = bench.roofline(_res(), 4)
    assert r["kernel"] == "reinit_xy" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    # two values of 4 bytes per grain voxel over 100 ms
    assert r["achieved"] == pytest.approx(2 * 4 * 3.0e10 / 0.1 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["avg_launch_ms"] == pytest.approx(0.5)
    assert r["alg_bytes_per_launch"] == pytest.approx(2 * 4 * 3.0e10 / 200)
    assert set(r["per_kernel"]) == {"conv_xy", "compare", "reinit_xy", "reinit_z"}


def test_roofline_counts_the_correction_and_the_jacobi_sweeps():
    r = bench.roofline(_res(physics=True), 4)
    # the re-initialization carries the ID-field: 8 more bytes per grain voxel
    assert r["achieved"] == pytest.approx((2 * 4 + 8) * 3.0e10 / 0.1 / 1e9)
    res = _res(sweeps=16)
    res["kernels"]["reinit_sweep"] = dict(ms=400.0, launches=3200, voxels=3.0e10)
    r = bench.roofline(res, 4)
    assert r["kernel"] == "reinit_sweep"
    assert r["achieved"] == pytest.approx(2 * 16 * 4 * 3.0e10 / 0.4 / 1e9)


def test_recorded_traffic_follows_the_sources(monkeypatch):
    path = os.path.join(ROOT, "profiles", "traffic_reinit_xy_3d256_8000g_fp32.md")
    fields = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ":" in line:
                a, b = line[2:].split(":", 1)
                fields[a.strip()] = b.strip().strip("`")
    got = bench.recorded_traffic("reinit_xy", "fp32", "3d256_8000g")
    if fields["source_sha256"] == bench.source_digest():
        assert got == float(fields["hbm_bytes_per_launch"])
    else:
        assert got is None
    assert bench.recorded_traffic("reinit_xy", "fp32", "no_such_workload") is None
    monkeypatch.setattr(bench, "source_digest", lambda: "0" * 64)
    assert bench.recorded_traffic("reinit_xy", "fp32", "3d256_8000g") is None


@pytest.mark.parametrize("dim,W", [(2, 6.0), (3, 8.0), (3, 5.5), (2, 16.0)])
def test_euclid_sweep_count(dim, W):
    K = bench.euclid_sweeps(dim, W)
    assert K % 2 == 0 and K >= math.ceil(math.sqrt(dim) * W) + 1 and K <= math.ceil(math.sqrt(dim) * W) + 2
