"""Host-side parts of bench.py: the one-GPU contract, the gate on the counted
HBM traffic (reported only while the kernel sources match the profile) and
the sweep point generators."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_counted_traffic_follows_the_kernel_sources(monkeypatch, tmp_path):
    t = bench.counted_traffic("num_window", "rmat20")
    # the committed counter summary, while the kernels are the ones it measured
    assert t is None or t > 3e11
    extra = tmp_path / "changed.hip"
    extra.write_text("// a different kernel source\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", bench.KERNEL_SOURCES + (str(extra),))
    assert bench.counted_traffic("num_window", "rmat20") is None
    assert bench.counted_traffic("no_such_kernel", "rmat20") is None


@pytest.mark.parametrize("name,first", [
    ("sweep_density", "er s16 ef2 unsorted"),
    ("sweep_size", "er s7 ef16 unsorted"),
])
def test_sweep_points(name, first):
    label, A, B, srt, params = next(bench._sweep_points(name, 1))
    assert label == first and A is B and srt is False
    assert A.nrows == 1 << params["scale"]
    assert A.nnz == A.nrows * params["ef"]             # ER rows hold exactly ef distinct columns
