"""Host logic of bench.py (CPU): the committed counter summaries are read only
while the kernel sources they hash are unchanged, and the JSON contract's
single-GPU rule."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _write_summary(tmp_path, src_text, digest=None):
    import hashlib
    src = tmp_path / "k.hip"
    src.write_text(src_text)
    h = hashlib.sha256(src.read_bytes()).hexdigest()[:16] if digest is None else digest
    prof = tmp_path / "profiles"
    prof.mkdir(exist_ok=True)
    (prof / "fp64_toy.md").write_text(
        "# toy\n\n- fp64_ops_per_launch.k_a: 1000\n- fp64_ops_per_launch.k_b: 24\n"
        f"- source: k.hip\n- source_sha256_16: {h}\n")
    return src


def test_recorded_fields_and_hash_guard(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    src = _write_summary(tmp_path, "kernel v1\n")
    rec = bench.recorded("fp64_toy")
    assert rec is not None and rec["path"] == os.path.join("profiles", "fp64_toy.md")
    assert bench.recorded_sum(rec, "fp64_ops_per_launch", ["k_a", "k_b"]) == 1024.0
    assert bench.recorded_sum(rec, "fp64_ops_per_launch", ["k_a", "k_c"]) is None
    src.write_text("kernel v2\n")  # the source changed since the counters were taken
    assert bench.recorded("fp64_toy") is None
    assert bench.recorded("fp64_missing") is None


def test_counter_rate_uses_group_kernels(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _write_summary(tmp_path, "kernel\n")

    class W:  # a workload of the fused path (n_big <= 64)
        name = "toy"
        params = {"n_big": 10, "n_small": 100}

    bench.GROUP_KERNELS[("toy_group", True)] = ["k_a", "k_b"]
    try:
        r = bench.counter_rate(W, "toy_group", 1e-6)
    finally:
        del bench.GROUP_KERNELS[("toy_group", True)]
    assert r["fp64_ops_per_launch"] == 1024.0
    assert r["achieved"] == pytest.approx(1024.0 / 1e-6 / 1e12)
    assert r["frac"] == pytest.approx(1024.0 / 1e-6 / bench.PEAK_FP64)
    assert bench.counter_rate(W, "no_such_group", 1e-6) is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode != 0 and "one GPU" in p.stderr
