"""Independent references used to pin the oracle (tests only)."""
from __future__ import annotations

import functools
import importlib.util
import os
import subprocess
import tempfile

import numpy as np

_HARNESS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "harness",
                        "philox_torch_ref.cpp")


@functools.lru_cache(maxsize=1)
def torch_philox_exe() -> str:
    spec = importlib.util.find_spec("torch")
    inc = os.path.join(list(spec.submodule_search_locations)[0], "include")
    out = os.path.join(tempfile.mkdtemp(prefix="skref_"), "philox_ref")
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", inc, _HARNESS, "-o", out], check=True)
    return out


def torch_philox(pairs) -> np.ndarray:
    """pairs: iterable of (key[2], ctr[4]) -> uint32 array (len, 4)."""
    lines = "".join("%x %x %x %x %x %x\n" % (k[0] & 0xFFFFFFFF, k[1] & 0xFFFFFFFF,
                                               c[0] & 0xFFFFFFFF, c[1] & 0xFFFFFFFF,
                                               c[2] & 0xFFFFFFFF, c[3] & 0xFFFFFFFF)
                    for k, c in pairs)
    res = subprocess.run([torch_philox_exe()], input=lines, capture_output=True, text=True,
                         check=True)
    rows = [[int(t, 16) for t in ln.split()] for ln in res.stdout.strip().splitlines()]
    return np.array(rows, dtype=np.uint32).reshape(-1, 4)


def words_for(seed: int, g: int, j: int) -> np.ndarray:
    """Generator words for row group g of S column j (counter (g, j_lo, j_hi, 0))."""
    return torch_philox([((seed & 0xFFFFFFFF, seed >> 32),
                          (g, j & 0xFFFFFFFF, j >> 32, 0))])[0]


def box_muller_f64(xe: np.ndarray, xo: np.ndarray):
    """FP64 libm Box-Muller on the same uniforms the FP32 transform uses:
    u1 = ((xe>>8)+1) 2^-24 in (0,1], u2 = (xo>>8) 2^-24 in [0,1)."""
    u1 = ((xe.astype(np.uint64) >> 8) + 1).astype(np.float64) * 2.0 ** -24
    u2 = (xo.astype(np.uint64) >> 8).astype(np.float64) * 2.0 ** -24
    r = np.sqrt(-2.0 * np.log(u1))
    return r * np.cos(2 * np.pi * u2), r * np.sin(2 * np.pi * u2), r
