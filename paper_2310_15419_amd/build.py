"""Build libsketch.so (HIP, gfx950) in-tree with hipcc.

Flags: no FP contraction and IEEE-rounded FP32 division/square root (the S
generator's FP32 sequence must round exactly as written); packed-FP32 VALU
instructions disabled; the hot kernels use FP32 FMA explicitly.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsketch.so")
SOURCES = [os.path.join(CSRC, "sk_lib.hip")]
HEADERS = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))] + \
    [os.path.join(ROOT, "include", "sketch.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         "-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into ``libsketch.so`` (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed")
    os.replace(tmp, LIB)
    return LIB


def asm(out_dir: str) -> None:
    """Write the device assembly (for inspecting the generated code)."""
    os.makedirs(out_dir, exist_ok=True)
    cmd = [HIPCC, *[f for f in FLAGS if f not in ("-shared", "-fPIC")], "--cuda-device-only",
           "-S", "-o", os.path.join(out_dir, "sk_lib.s"), *SOURCES]
    subprocess.run(cmd, check=True)


if __name__ == "__main__":
    print(build(verbose=True))
