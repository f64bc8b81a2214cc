"""Host logic of bench.py (no GPU): the one-GPU contract, the algorithmic
bytes of the stream-collide, and the HBM traffic taken from the committed
counter summary only while the kernel source it was measured on is unchanged."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout.strip()


def test_copy_ceiling_is_null_without_a_gpu():
    import torch
    if torch.cuda.is_available():
        return
    assert bench.copy_ceiling(1000) is None


def test_cpu_model_is_a_name_or_none():
    m = bench.cpu_model()
    assert m is None or (isinstance(m, str) and m)


def test_algorithmic_bytes_per_node():
    # 19 populations read and 19 written: 4 bytes each (FP32), 2 bytes (FP16 / BF16)
    assert bench.bytes_per_node(0) == 152
    assert bench.bytes_per_node(1) == 76 and bench.bytes_per_node(2) == 76


def test_traffic_follows_the_kernel_source(monkeypatch):
    recorded = None
    for line in open(bench.PMC_SUMMARY):
        if line.startswith("kernel_source_sha256_16"):
            recorded = line.split("=", 1)[1].strip()
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: recorded)
    t = bench.traffic_from_profile()
    assert t is not None and 9.0e8 < t < 1.1e9  # ~961.6e6 algorithmic bytes per launch
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "0" * 16)  # the kernel changed since
    assert bench.traffic_from_profile() is None
