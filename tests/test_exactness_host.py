"""Host checks of three exactness arguments of the kernels: the division-free
minimum image (a threshold compare in place of floor(d / L + 0.5)) gives bit
for bit the result of the plain formula, checked on a host build of the same
header over many axis lengths, at and around both thresholds, at +-L/2, zero
and random offsets; and the fast metaball sum behind the flag decision stays
within its stated bound of the exact sum, and the FP32 first decision of
C >= L agrees with the exact one wherever it is taken."""
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


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")
def test_fast_metaball_sum_is_within_its_bound(tmp_path):
    """The flag decision evaluates C with refined reciprocals and falls back
    to exact quotients within 1e-12 of 1: the fast sum must stay within
    1e-13 C of the exact one near the surface, even from a reciprocal
    estimate much worse than the hardware's."""
    exe = tmp_path / "metaball_fast_check"
    src = os.path.join(ROOT, "tests", "native", "metaball_fast_check.cpp")
    subprocess.run(["g++", "-std=c++17", "-O2", "-ffp-contract=off", src, "-o", str(exe)],
                   check=True, capture_output=True, timeout=300)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")
def test_fp32_metaball_decision_agrees_with_the_exact_one(tmp_path):
    """Flagging and the link bracket first decide C >= L in FP32 (relative
    coordinates, hardware reciprocal) and keep that decision only when the
    FP32 sum clears L by its error bound: over random bodies, at points near
    the surface down to 1e-8 relative, near control points and on lattice
    points, every kept decision must equal the exact one, and nearly every
    lattice point must be decided in FP32 (the speed-up)."""
    exe = tmp_path / "metaball_f32_check"
    src = os.path.join(ROOT, "tests", "native", "metaball_f32_check.cpp")
    subprocess.run(["g++", "-std=c++17", "-O2", "-ffp-contract=off", src, "-o", str(exe)],
                   check=True, capture_output=True, timeout=300)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
    assert " 0 disagreements" in r.stdout
