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


def test_oracle_rate_runs_a_bounded_sample_on_the_requested_threads():
    """The CPU baseline's sampler: at least the minimum number of coupled
    oracle steps, a positive rate, and the oracle's thread count set back."""
    import oracle
    import workloads

    cfg = workloads.small_settling(n=16, nz=24, R=3.0)
    nt = oracle.threads()
    v, steps, t_init = bench._oracle_rate(cfg, 0.0, min_steps=2)
    assert steps == 2 and v > 0.0 and t_init >= 0.0
    oracle.set_threads(1)
    try:
        assert oracle.threads() == 1
        v1, s1, _ = bench._oracle_rate(cfg, 0.0, min_steps=1)
        assert s1 == 1 and v1 > 0.0
    finally:
        oracle.set_threads(nt)
    assert oracle.threads() == nt
