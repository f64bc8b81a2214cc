"""The division-free minimum image used by the kernels (a threshold compare
in place of floor(d / L + 0.5)) gives bit for bit the result of the plain
formula: a host build of the same header checked over many axis lengths,
at and around both thresholds, at +-L/2 and zero, and at random offsets."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not found")
def test_min_image_thresholds_are_exact(tmp_path):
    exe = tmp_path / "min_image_check"
    src = os.path.join(ROOT, "tests", "native", "min_image_check.cpp")
    subprocess.run(["hipcc", "-std=c++17", "-O2", "-x", "hip", "--offload-arch=gfx950", src, "-o", str(exe)],
                   check=True, capture_output=True, timeout=300)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
    assert " 0 mismatches" in r.stdout
