"""ctypes binding of libsketch.so (argument marshalling only).

Device memory and streams come from PyTorch; every step of the computation
runs in the library's HIP kernels.  Loading fails loudly when the library is
missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsketch.so")

RADEMACHER, UNIFORM, GAUSSIAN = 0, 1, 2
DISTS = {"rademacher": RADEMACHER, "pm1": RADEMACHER, "uniform": UNIFORM, "gaussian": GAUSSIAN}
F64, F32, BF16 = 0, 1, 2
PREC_F32, PREC_BF16, PREC_FP8 = 0, 1, 2


class SkCsc(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("colptr", ctypes.c_void_p), ("rowidx", ctypes.c_void_p),
                ("vals", ctypes.c_void_p), ("vtype", ctypes.c_int32)]


class SkTuning(ctypes.Structure):
    _fields_ = [("rows_per_block", ctypes.c_int32), ("splits", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("dense_min_pct", ctypes.c_int32),
                ("phases", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
                ("col_split", ctypes.c_int32), ("row_pad", ctypes.c_int32)]


class SketchError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {status_string(code)} ({code})")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first "
                               "(python -m paper_2310_15419_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        P, vp, i32, i64, u64 = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, \
            ctypes.c_uint64
        L.sk_status_string.argtypes = [ctypes.c_int]
        L.sk_status_string.restype = ctypes.c_char_p
        L.sk_variant_count.restype = ctypes.c_int
        L.sk_sketch_workspace.argtypes = [P(SkCsc), i64, i32, i32, P(SkTuning), P(ctypes.c_size_t)]
        L.sk_sketch.argtypes = [P(SkCsc), i64, i64, i32, u64, i32, P(SkTuning), vp, i64, vp,
                                ctypes.c_size_t, vp]
        L.sk_sketch_status.argtypes = [vp, vp, P(i64), P(i64)]
        L.sk_materialize_s.argtypes = [i64, i64, i64, i64, i32, u64, vp, i64, vp]
        L.sk_autotune.argtypes = [P(SkCsc), i64, i32, P(SkTuning)]
        L.sk_sketch_batched_workspace.argtypes = [i32, P(SkCsc), P(i64), P(i32), i32, P(SkTuning),
                                                  P(ctypes.c_size_t)]
        L.sk_sketch_batched.argtypes = [i32, P(SkCsc), P(i64), P(i32), P(u64), i32, P(SkTuning),
                                        P(vp), P(i64), vp, ctypes.c_size_t, vp]
        L.sk_sketch_batched_plan.argtypes = [i32, P(SkCsc), P(i64), P(i32), i32, P(SkTuning),
                                             P(SkTuning)]
        L.sk_sketch_batched_status.argtypes = [vp, i32, vp, P(i32)]
        L.sk_rng_tables.argtypes = [vp, vp, vp, vp]
        L.sk_rng_tables.restype = None
        for name in ("sk_sketch_workspace", "sk_sketch", "sk_sketch_status", "sk_materialize_s",
                     "sk_autotune", "sk_sketch_batched_workspace", "sk_sketch_batched",
                     "sk_sketch_batched_plan", "sk_sketch_batched_status"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(code: int) -> str:
    return lib().sk_status_string(code).decode()


def _check(code: int, what: str):
    if code != 0:
        raise SketchError(code, what)


def _dist(dist) -> int:
    return DISTS[dist] if isinstance(dist, str) else int(dist)


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _tuning(tune):
    if tune is None:
        return None
    if isinstance(tune, SkTuning):
        return ctypes.byref(tune)
    t = SkTuning(int(tune.get("rows_per_block", 0)), int(tune.get("splits", 0)),
                 int(tune.get("variant", 0)), int(tune.get("dense_min_pct", 0)),
                 int(tune.get("phases", 0)), int(tune.get("tile_rows", 0)),
                 int(tune.get("col_split", 0)), int(tune.get("row_pad", 0)))
    return ctypes.byref(t)


@dataclasses.dataclass
class DeviceCsc:
    """A CSC matrix whose arrays are device tensors (the library's input)."""
    m: int
    n: int
    colptr: "object"
    rowidx: "object"
    vals: "object"

    @property
    def nnz(self) -> int:
        return int(self.rowidx.numel())

    @property
    def vtype(self) -> int:
        import torch
        return {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}[self.vals.dtype]

    def c_struct(self) -> SkCsc:
        return SkCsc(self.m, self.n, self.nnz, self.colptr.data_ptr(),
                     self.rowidx.data_ptr() if self.nnz else None,
                     self.vals.data_ptr() if self.nnz else None, self.vtype)

    @staticmethod
    def from_host(A, device="cuda", dtype=None) -> "DeviceCsc":
        """Upload a host CSC (``inputs.Csc``) to the device."""
        import torch
        vals = A.vals if dtype is None else A.vals.astype(dtype)
        tv = torch.from_numpy(np.ascontiguousarray(vals))
        return DeviceCsc(A.m, A.n,
                         torch.from_numpy(np.ascontiguousarray(A.colptr, np.int64)).to(device),
                         torch.from_numpy(np.ascontiguousarray(A.rowidx, np.int32)).to(device),
                         tv.to(device))


def workspace_bytes(A: DeviceCsc, d: int, dist, prec: int = PREC_F32, tune=None) -> int:
    out = ctypes.c_size_t()
    c = A.c_struct()
    _check(lib().sk_sketch_workspace(ctypes.byref(c), d, _dist(dist), prec, _tuning(tune),
                                     ctypes.byref(out)), "sk_sketch_workspace")
    return int(out.value)


def alloc_workspace(nbytes: int, device="cuda"):
    import torch
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def sketch_into(A: DeviceCsc, d: int, dist, seed: int, out, ws, row0: int = 0,
                prec: int = PREC_F32, tune=None, stream=None, ld: int | None = None) -> None:
    """Enqueue A_hat = S[row0:row0+d] A into ``out`` (FP32, column-major d x n with
    leading dimension ld, i.e. a tensor of shape (n, ld) in row-major terms)."""
    c = A.c_struct()
    ld = d if ld is None else ld
    _check(lib().sk_sketch(ctypes.byref(c), row0, d, _dist(dist), seed, prec, _tuning(tune),
                           out.data_ptr(), ld, ws.data_ptr(), ws.numel(), _stream(stream)),
           "sk_sketch")


def sketch(A: DeviceCsc, d: int, dist, seed: int, row0: int = 0, prec: int = PREC_F32,
           tune=None, stream=None, check: bool = True):
    """A_hat = S[row0:row0+d, :] @ A as a torch FP32 tensor of shape (d, n)."""
    import torch
    ws = alloc_workspace(workspace_bytes(A, d, dist, prec, tune), A.colptr.device)
    out = torch.empty((A.n, d), dtype=torch.float32, device=A.colptr.device)
    sketch_into(A, d, dist, seed, out, ws, row0, prec, tune, stream)
    if check:
        st = sketch_status(ws, stream)
        _check(st["status"], "sk_sketch (device validation)")
    return out.t()


def sketch_status(ws, stream=None) -> dict:
    R = ctypes.c_int64()
    nb = ctypes.c_int64()
    code = lib().sk_sketch_status(ctypes.c_void_p(ws.data_ptr()), _stream(stream),
                                  ctypes.byref(R), ctypes.byref(nb))
    return {"status": int(code), "nonempty_rows": int(R.value), "row_blocks": int(nb.value)}


def materialize_s(row0: int, d: int, col0: int, ncols: int, dist, seed: int, stream=None):
    """S[row0:row0+d, col0:col0+ncols] from the device generator (torch FP32, (d, ncols))."""
    import torch
    out = torch.empty((ncols, d), dtype=torch.float32, device="cuda")
    _check(lib().sk_materialize_s(row0, d, col0, ncols, _dist(dist), seed, out.data_ptr(), d,
                                  _stream(stream)), "sk_materialize_s")
    return out.t()


def rng_tables() -> dict:
    lc = np.empty(5, np.float32)
    sc = np.empty(7, np.float32)
    cc = np.empty(8, np.float32)
    mc = np.empty(3, np.float32)
    lib().sk_rng_tables(lc.ctypes.data, sc.ctypes.data, cc.ctypes.data, mc.ctypes.data)
    return {"log": lc, "sin": sc, "cos": cc, "misc": mc}


def variant_count() -> int:
    return int(lib().sk_variant_count())


def autotune(A: DeviceCsc, d: int, dist) -> dict:
    """The tuning the library picks for this shape."""
    t = SkTuning()
    c = A.c_struct()
    _check(lib().sk_autotune(ctypes.byref(c), d, _dist(dist), ctypes.byref(t)), "sk_autotune")
    return tuning_dict(t)


def tuning_dict(t: SkTuning) -> dict:
    return {f[0]: int(getattr(t, f[0])) for f in SkTuning._fields_}


class Batch:
    """Marshalled arguments of one batched call (host arrays of the C ABI)."""

    def __init__(self, mats, ds, dists, seeds, tunes=None, prec: int = PREC_F32):
        n = len(mats)
        self.count = n
        self.mats = mats
        self.c_mats = (SkCsc * n)(*[A.c_struct() for A in mats])
        self.c_d = (ctypes.c_int64 * n)(*[int(x) for x in ds])
        self.c_dist = (ctypes.c_int32 * n)(*[_dist(x) for x in dists])
        self.c_seed = (ctypes.c_uint64 * n)(*[int(x) for x in seeds])
        self.c_tune = None
        if tunes is not None:
            self.c_tune = (SkTuning * n)(*[SkTuning(*[int(t.get(f[0], 0)) for f in SkTuning._fields_])
                                          for t in tunes])
        self.prec = prec
        self.ds = [int(x) for x in ds]

    def workspace_bytes(self) -> int:
        out = ctypes.c_size_t()
        _check(lib().sk_sketch_batched_workspace(self.count, self.c_mats, self.c_d, self.c_dist,
                                                 self.prec, self.c_tune, ctypes.byref(out)),
               "sk_sketch_batched_workspace")
        return int(out.value)

    def plan(self) -> list:
        out = (SkTuning * self.count)()
        _check(lib().sk_sketch_batched_plan(self.count, self.c_mats, self.c_d, self.c_dist,
                                            self.prec, self.c_tune, out), "sk_sketch_batched_plan")
        return [tuning_dict(t) for t in out]

    def run(self, outs, ws, stream=None) -> None:
        """outs[i]: FP32 tensor of shape (n_i, d_i) (column-major d_i x n_i)."""
        ptrs = (ctypes.c_void_p * self.count)(*[o.data_ptr() for o in outs])
        lds = (ctypes.c_int64 * self.count)(*self.ds)
        _check(lib().sk_sketch_batched(self.count, self.c_mats, self.c_d, self.c_dist, self.c_seed,
                                       self.prec, self.c_tune, ptrs, lds, ws.data_ptr(), ws.numel(),
                                       _stream(stream)), "sk_sketch_batched")

    def status(self, ws, stream=None) -> list:
        st = (ctypes.c_int32 * self.count)()
        lib().sk_sketch_batched_status(ctypes.c_void_p(ws.data_ptr()), self.count, _stream(stream),
                                       st)
        return list(st)


EXPORTED = ["sk_status_string", "sk_variant_count", "sk_sketch_workspace", "sk_sketch",
            "sk_sketch_status", "sk_materialize_s", "sk_rng_tables", "sk_autotune",
            "sk_sketch_batched_workspace", "sk_sketch_batched", "sk_sketch_batched_plan",
            "sk_sketch_batched_status"]
