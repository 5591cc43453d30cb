"""CPU oracle for the sketch A_hat = S A (paper Sec. I-A, eq. (1)).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this module; the product path must not.  The C
file ``sk_oracle.c`` holds the arithmetic (FP64 accumulation, explicit S);
this module only marshals arguments and builds the shared object.

Pinned functions (each is checked in ``tests/test_oracle_*.py`` against
something other than itself):
  philox        -- against two independent Philox4x32-10 engines (PyTorch's
                   header engine, compiled into a test harness; rocRAND's
                   host generator through its C API)
  s_entry / materialize_s -- against the generator words (independent Philox)
                   for +-1 and (-1,1) exactly; Gaussian against FP64 libm
                   Box-Muller
  sketch        -- brute force, identity blocks, linearity, concatenation,
                   E[A_hat^T A_hat] = d sigma^2 A^T A, subspace embedding
  parity        -- error measures only (no part of the method); pinned by a
                   brute-force recomputation on a small case
  ls_error / sap_solve_reference -- numpy least squares on dense inputs
  sap_svd_reference -- the minimum-norm solution of exactly rank-deficient
                   stand-ins (orthogonality to the known null vectors, numpy's
                   minimum-norm lstsq), the drop threshold from both sides,
                   agreement with the QR form on full-rank input
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sk_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD, "libskoracle.so")

RADEMACHER, UNIFORM, GAUSSIAN = 0, 1, 2
DIST_NAMES = {"rademacher": RADEMACHER, "pm1": RADEMACHER, "uniform": UNIFORM,
              "gaussian": GAUSSIAN}
SIGMA2 = {RADEMACHER: 1.0, UNIFORM: 1.0 / 3.0, GAUSSIAN: 1.0}


def build(force: bool = False) -> str:
    """Compile the C oracle (gcc, OpenMP, no FP contraction, no fast-math)."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        L.or_philox4x32_10.argtypes = [P(ctypes.c_uint32), P(ctypes.c_uint32), P(ctypes.c_uint32)]
        L.or_s_entry.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64]
        L.or_s_entry.restype = ctypes.c_double
        L.or_materialize_s.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                       ctypes.c_int64, ctypes.c_int]
        L.or_sketch.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                ctypes.c_int64]
        L.or_sketch.restype = ctypes.c_int
        L.or_gauss_words.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]
        L.or_tables.argtypes = [ctypes.c_void_p] * 4
        L.or_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _dist(dist) -> int:
    if isinstance(dist, str):
        return DIST_NAMES[dist]
    return int(dist)


def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 of one 128-bit counter (4 words) under a 64-bit key (2 words)."""
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def s_entry(dist, seed: int, i: int, j: int) -> float:
    """S(i, j): global S row i, S column j (= A row j)."""
    return lib().or_s_entry(_dist(dist), seed, i, j)


def materialize_s(dist, seed: int, row0: int, d: int, col0: int, ncols: int,
                  threads: int = 0) -> np.ndarray:
    """S[row0:row0+d, col0:col0+ncols] as an FP64 array (exact widening of FP32)."""
    out = np.empty((d, ncols), dtype=np.float64, order="F")
    lib().or_materialize_s(_dist(dist), seed, row0, d, col0, ncols,
                           out.ctypes.data, d, threads)
    return out


def sketch(m: int, n: int, colptr, rowidx, vals, d: int, dist, seed: int,
           row0: int = 0, panel: int = 0, threads: int = 0) -> np.ndarray:
    """A_hat = S[row0:row0+d, :] @ A in FP64 (column-major d x n).

    ``panel`` = number of S columns materialised at once (0: a panel sized to
    about 256 MB of FP64, or the whole S if that is smaller)."""
    colptr = np.ascontiguousarray(colptr, dtype=np.int64)
    rowidx = np.ascontiguousarray(rowidx, dtype=np.int32)
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    if panel <= 0:
        panel = max(1, min(m, (256 << 20) // (8 * d)))
    out = np.empty((d, n), dtype=np.float64, order="F")
    rc = lib().or_sketch(m, n, colptr.ctypes.data, rowidx.ctypes.data, vals.ctypes.data,
                         row0, d, _dist(dist), seed, panel, threads, out.ctypes.data, d)
    if rc != 0:
        raise ValueError(f"oracle sketch rejected the input (code {rc})")
    return out


def gauss_words(xe, xo):
    """The FP32 Box-Muller transform applied to explicit word pairs."""
    xe = np.ascontiguousarray(xe, dtype=np.uint32)
    xo = np.ascontiguousarray(xo, dtype=np.uint32)
    z0 = np.empty(xe.shape, dtype=np.float32)
    z1 = np.empty(xe.shape, dtype=np.float32)
    lib().or_gauss_words(xe.size, xe.ctypes.data, xo.ctypes.data, z0.ctypes.data, z1.ctypes.data)
    return z0, z1


def tables():
    """The oracle's FP32 coefficient tables (log series, sine, cosine, misc)."""
    lc = np.empty(5, np.float32)
    sc = np.empty(7, np.float32)
    cc = np.empty(8, np.float32)
    mc = np.empty(3, np.float32)
    lib().or_tables(lc.ctypes.data, sc.ctypes.data, cc.ctypes.data, mc.ctypes.data)
    return {"log": lc, "sin": sc, "cos": cc, "misc": mc}


# largest |S| entry per distribution: +-1, the open interval (-1,1), and the
# largest radius the Gaussian transform can produce, sqrt(-2 ln 2^-24)
S_MAX = {RADEMACHER: 1.0, UNIFORM: 1.0, GAUSSIAN: float(np.sqrt(48.0 * np.log(2.0)))}
# element-wise bar of the FP32 path, relative to the scale of the terms summed
# into the element (see ``parity``)
ELEM_TOL = 2.0 ** -20


def parity(got, ref, colptr, vals, dist) -> dict:
    """Errors of a sketch ``got`` (d x n) against the oracle's ``ref``:
    normwise ||got - ref||_F / ||ref||_F, the largest per-column relative
    2-norm error, and the largest element-wise error scaled by the size of
    the terms summed into that element, |got_ik - ref_ik| / (max|S| sum_j
    |a_jk|) (an FP32 sum of K terms is off by at most about K u of that
    scale, and typically by sqrt(K) u)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if got.shape != ref.shape:
        raise ValueError(f"shape {got.shape} != {ref.shape}")
    diff = np.abs(got - ref)
    rnorm = np.linalg.norm(ref)
    normwise = float(np.linalg.norm(diff) / rnorm) if rnorm > 0 else float(np.linalg.norm(diff))
    cref = np.linalg.norm(ref, axis=0)
    cdiff = np.linalg.norm(diff, axis=0)
    col = np.where(cref > 0, cdiff / np.where(cref > 0, cref, 1.0), cdiff)
    colptr = np.asarray(colptr, dtype=np.int64)
    n = colptr.size - 1
    owner = np.repeat(np.arange(n), np.diff(colptr))
    scale = np.bincount(owner, weights=np.abs(np.asarray(vals, dtype=np.float64)), minlength=n)
    scale = scale * S_MAX[_dist(dist)]
    elem = np.where(scale > 0, diff / np.where(scale > 0, scale, 1.0), diff)
    return {"normwise": normwise, "max_col": float(col.max()) if col.size else 0.0,
            "max_elem_scaled": float(elem.max()) if elem.size else 0.0,
            "nonfinite": int(np.count_nonzero(~np.isfinite(got)))}


def max_threads() -> int:
    return lib().or_max_threads()


from .lsq import SVD_DROP, ls_error, sap_solve_reference, sap_svd_reference  # noqa: E402,F401
