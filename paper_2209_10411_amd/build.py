"""Builds libmidelbm.so (HIP for gfx950) in this directory with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, "csrc", "kernels.hip"), os.path.join(HERE, "csrc", "mlp.hip"),
       os.path.join(HERE, "csrc", "api.cpp"), os.path.join(HERE, "csrc", "copy_probe.hip"),
       os.path.join(HERE, "csrc", "mifit.hip"), os.path.join(HERE, "csrc", "shape.hip")]
LIB = os.path.join(HERE, "libmidelbm.so")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # no packed FP32 instructions (v_pk_*_f32) in device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def build(verbose: bool = False) -> str:
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = ["hipcc", *FLAGS, "-o", tmp, *SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
