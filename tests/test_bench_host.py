"""Host-side logic of bench.py (no GPU): the one-GPU guard, the algorithmic
work and byte counts the roofline figures divide by, and the rule that a
counter-measured traffic figure applies only to the workload and kernel
sources it was taken on."""
import os
import subprocess
import sys

import pytest

from paper_1411_1702_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_of_the_update_launch():
    # Robertson: 124 bytes per particle (gathered x 12, theta 24, predictor
    # likelihood 8; written x 12, theta 24, weight 8; the drawn-ahead normals
    # 24; the ancestor's prefix 8; the ancestor written 4)
    assert bench.algorithmic_bytes(inputs.robertson(1 << 17, 5)) == 124 << 17
    # chain: 2 (64 + 96 + 8) + 4 (12 + 16) + 8 + 4
    assert bench.algorithmic_bytes(inputs.chain16(1024, 5)) == 460 * 1024
    ad = inputs.advdiff(64, 2, seed=0, n=20)
    assert bench.algorithmic_bytes(ad) == (8 * 361 + 2 * 8 * 5 + 3 * 8 + 4) * 64


def test_advdiff_flops_count_transforms_and_recurrences():
    p20 = inputs.advdiff(64, 2, seed=0, n=20)
    nt, M = 19, p20.substeps
    modes = nt * (nt // 2 + 1)
    tr = 12 * nt * nt * (nt // 2 + 1)
    assert bench.advdiff_flops(p20, False) == 2 * tr + M * modes * 25
    assert bench.advdiff_flops(p20, True) == (2 + M) * tr + M * modes * 45
    # the O(nt^3) transforms dominate: doubling the side multiplies by ~8
    p40 = inputs.advdiff(64, 2, seed=0, n=40)
    r = bench.advdiff_flops(p40, True) / bench.advdiff_flops(p20, True)
    assert 7.0 < r < 9.5


def test_kernel_source_hash_is_stable_and_short():
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    assert bench.kernel_source_hash() == h


def test_traffic_figure_only_for_its_workload(monkeypatch):
    prob = inputs.robertson(1 << 17, 5)
    monkeypatch.setattr(bench, "TRAFFIC", {bench.kernel_source_hash(): {
        "fetch_kib": 100.0, "write_kib": 50.0, "fetch_scale": 2.0, "write_scale": 1.0}})
    assert bench.update_traffic_bytes(prob) == 1024.0 * (200.0 + 50.0)
    for change in ({"lmm": 1}, {"order": 3}, {"substeps": 10}, {"resampling": 1}):
        other = inputs.robertson(1 << 17, 5)
        for k, v in change.items():
            setattr(other, k, v)
        assert bench.update_traffic_bytes(other) is None, change
    assert bench.update_traffic_bytes(inputs.robertson(1 << 16, 5)) is None
    assert bench.update_traffic_bytes(inputs.chain16(1 << 17, 5)) is None
    # counters taken on other kernel sources do not apply
    monkeypatch.setattr(bench, "TRAFFIC", {"0" * 16: {
        "fetch_kib": 100.0, "write_kib": 50.0, "fetch_scale": 2.0, "write_scale": 1.0}})
    assert bench.update_traffic_bytes(prob) is None


def test_peaks_are_the_published_figures():
    assert bench.PEAK_VALU_NONPACKED == pytest.approx(78.6, abs=0.1)
    assert bench.PEAK_FP32_PUBLISHED == pytest.approx(157.3)
