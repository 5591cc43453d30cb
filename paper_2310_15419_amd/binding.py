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
                ("col_split", ctypes.c_int32), ("row_pad", ctypes.c_int32),
                ("count_rng", ctypes.c_int32), ("rng_mode", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("balance", ctypes.c_int32)]


class SapParams(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int64), ("dist", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("atol", ctypes.c_double), ("btol", ctypes.c_double),
                ("conlim", ctypes.c_double), ("iter_lim", ctypes.c_int32),
                ("method", ctypes.c_int32)]


class SapInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("istop", ctypes.c_int32),
                ("done", ctypes.c_int32), ("iter_lim", ctypes.c_int32),
                ("rnorm", ctypes.c_double), ("arnorm", ctypes.c_double),
                ("anorm", ctypes.c_double), ("acond", ctypes.c_double),
                ("xnorm", ctypes.c_double), ("bnorm", ctypes.c_double),
                ("test1", ctypes.c_double), ("test2", ctypes.c_double),
                ("test3", ctypes.c_double),
                ("rank", ctypes.c_int32), ("sweeps", ctypes.c_int32)]


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
        L.sk_sketch_noalloc.argtypes = [P(SkCsc), i64, i64, i32, u64, i32, P(SkTuning), vp, i64,
                                        vp]
        L.sk_sketch_status.argtypes = [vp, vp, P(i64), P(i64)]
        L.sk_sketch_rng_calls.argtypes = [vp, vp, P(ctypes.c_uint64)]
        L.sk_sketch_stored.argtypes = [P(SkCsc), i64, vp, i64, P(SkTuning), vp, i64, vp,
                                       ctypes.c_size_t, vp]
        L.sk_rng_throughput.argtypes = [i32, i32, i64, i32, u64, vp, vp]
        L.sk_sketch_colwise_workspace.argtypes = [P(SkCsc), i64, P(ctypes.c_size_t)]
        L.sk_sketch_colwise.argtypes = [P(SkCsc), i64, i64, i32, u64, vp, i64, vp,
                                        ctypes.c_size_t, vp]
        L.sk_sketch_colwise_f64.argtypes = [P(SkCsc), i64, i64, i32, u64, vp, i64, vp,
                                            ctypes.c_size_t, vp]
        L.sk_materialize_s.argtypes = [i64, i64, i64, i64, i32, u64, vp, i64, vp]
        L.sk_autotune.argtypes = [P(SkCsc), i64, i32, P(SkTuning)]
        L.sk_plan_info.argtypes = [P(SkCsc), i64, i32, i32, P(SkTuning), P(ctypes.c_double), i32]
        L.sk_autotune_workspace.argtypes = [P(SkCsc), i64, i32, i32, P(ctypes.c_size_t)]
        L.sk_autotune_measure.argtypes = [P(SkCsc), i64, i32, u64, i32, vp, i64, vp,
                                          ctypes.c_size_t, vp, P(SkTuning), P(ctypes.c_double)]
        L.sk_plan_cache_lookup.argtypes = [P(SkCsc), i64, i32, i32, P(SkTuning)]
        L.sk_plan_cache_clear.argtypes = []
        L.sk_plan_cache_clear.restype = None
        L.sk_sketch_batched_workspace.argtypes = [i32, P(SkCsc), P(i64), P(i32), i32, P(SkTuning),
                                                  P(ctypes.c_size_t)]
        L.sk_sketch_batched.argtypes = [i32, P(SkCsc), P(i64), P(i32), P(u64), i32, P(SkTuning),
                                        P(vp), P(i64), vp, ctypes.c_size_t, vp]
        L.sk_sketch_batched_plan.argtypes = [i32, P(SkCsc), P(i64), P(i32), i32, P(SkTuning),
                                             P(SkTuning)]
        L.sk_sketch_batched_status.argtypes = [vp, i32, vp, P(i32)]
        L.sk_rng_tables.argtypes = [vp, vp, vp, vp]
        L.sk_rng_tables.restype = None
        L.sk_qr_f64_workspace.argtypes = [i64, i64, P(ctypes.c_size_t)]
        L.sk_qr_f64.argtypes = [i64, i64, vp, i64, vp, i64, vp, ctypes.c_size_t, vp]
        L.sk_trinv_f64.argtypes = [i64, vp, i64, vp, i64, vp]
        L.sk_svd_f64_workspace.argtypes = [i64, i64, P(ctypes.c_size_t)]
        L.sk_svd_f64.argtypes = [i64, i64, vp, vp, vp, P(i32), vp, ctypes.c_size_t, vp]
        L.sk_sap_workspace.argtypes = [P(SkCsc), P(SapParams), P(ctypes.c_size_t)]
        L.sk_sap_begin.argtypes = [P(SkCsc), vp, P(SapParams), vp, ctypes.c_size_t, vp]
        L.sk_sap_iterate.argtypes = [P(SkCsc), P(SapParams), i32, vp, ctypes.c_size_t, vp]
        L.sk_sap_finish.argtypes = [P(SkCsc), P(SapParams), vp, vp, ctypes.c_size_t, vp]
        L.sk_sap_read_info.argtypes = [P(SkCsc), P(SapParams), vp, ctypes.c_size_t, vp,
                                       P(SapInfo)]
        for name in ("sk_sketch_workspace", "sk_sketch", "sk_sketch_noalloc", "sk_sketch_status",
                     "sk_sketch_rng_calls", "sk_sketch_stored", "sk_rng_throughput",
                     "sk_sketch_colwise_workspace", "sk_sketch_colwise",
                     "sk_sketch_colwise_f64", "sk_materialize_s",
                     "sk_autotune", "sk_plan_info", "sk_autotune_workspace",
                     "sk_autotune_measure", "sk_plan_cache_lookup",
                     "sk_sketch_batched_workspace", "sk_sketch_batched",
                     "sk_sketch_batched_plan", "sk_sketch_batched_status", "sk_qr_f64_workspace",
                     "sk_qr_f64", "sk_trinv_f64", "sk_svd_f64_workspace", "sk_svd_f64",
                     "sk_sap_workspace", "sk_sap_begin",
                     "sk_sap_iterate", "sk_sap_finish", "sk_sap_read_info"):
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
    unknown = set(tune) - {f[0] for f in SkTuning._fields_}
    if unknown:
        raise ValueError(f"unknown tuning fields {sorted(unknown)}")
    t = SkTuning(**{k: int(v) for k, v in tune.items()})
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


NOALLOC_SCRATCH_BYTES = 64 << 20  # SK_NOALLOC_SCRATCH_BYTES


def sketch_noalloc_into(A: DeviceCsc, d: int, dist, seed: int, out, row0: int = 0,
                        prec: int = PREC_F32, tune=None, stream=None,
                        ld: int | None = None) -> None:
    """sk_sketch_noalloc: like ``sketch_into`` with the library's fixed device
    array as the workspace (no workspace argument, nothing allocated)."""
    c = A.c_struct()
    ld = d if ld is None else ld
    _check(lib().sk_sketch_noalloc(ctypes.byref(c), row0, d, _dist(dist), seed, prec,
                                   _tuning(tune), out.data_ptr(), ld, _stream(stream)),
           "sk_sketch_noalloc")


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


def sketch_stored_into(A: DeviceCsc, S, out, ws, tune=None, stream=None) -> None:
    """sk_sketch_stored: A_hat = S A with S given (a torch FP32 tensor of shape
    (m, lds), i.e. column-major d x m with leading dimension lds)."""
    c = A.c_struct()
    d = out.shape[1]
    _check(lib().sk_sketch_stored(ctypes.byref(c), d, S.data_ptr(), S.shape[1], _tuning(tune),
                                  out.data_ptr(), d, ws.data_ptr(), ws.numel(), _stream(stream)),
           "sk_sketch_stored")


def colwise_workspace_bytes(A: DeviceCsc, d: int) -> int:
    out = ctypes.c_size_t()
    c = A.c_struct()
    _check(lib().sk_sketch_colwise_workspace(ctypes.byref(c), d, ctypes.byref(out)),
           "sk_sketch_colwise_workspace")
    return int(out.value)


def sketch_colwise_into(A: DeviceCsc, d: int, dist, seed: int, out, ws, row0: int = 0,
                        stream=None) -> None:
    """sk_sketch_colwise (the Algorithm 3 loop order) into ``out`` (n, d)."""
    c = A.c_struct()
    _check(lib().sk_sketch_colwise(ctypes.byref(c), row0, d, _dist(dist), seed, out.data_ptr(),
                                   d, ws.data_ptr(), ws.numel(), _stream(stream)),
           "sk_sketch_colwise")


def sketch_colwise_f64(A: DeviceCsc, d: int, dist, seed: int, row0: int = 0,
                       check: bool = True):
    """sk_sketch_colwise_f64: A_hat in FP64 (the same S), torch FP64 (d, n)."""
    import torch
    ws = alloc_workspace(colwise_workspace_bytes(A, d), A.colptr.device)
    out = torch.empty((A.n, d), dtype=torch.float64, device=A.colptr.device)
    c = A.c_struct()
    _check(lib().sk_sketch_colwise_f64(ctypes.byref(c), row0, d, _dist(dist), seed,
                                       out.data_ptr(), d, ws.data_ptr(), ws.numel(),
                                       _stream(None)), "sk_sketch_colwise_f64")
    if check:
        _check(sketch_status(ws)["status"], "sk_sketch_colwise_f64 (device validation)")
    return out.t()


def sketch_colwise(A: DeviceCsc, d: int, dist, seed: int, row0: int = 0, check: bool = True):
    """A_hat in the Algorithm 3 loop order, as a torch FP32 tensor of shape (d, n)."""
    import torch
    ws = alloc_workspace(colwise_workspace_bytes(A, d), A.colptr.device)
    out = torch.empty((A.n, d), dtype=torch.float32, device=A.colptr.device)
    sketch_colwise_into(A, d, dist, seed, out, ws, row0)
    if check:
        _check(sketch_status(ws)["status"], "sk_sketch_colwise (device validation)")
    return out.t()


def rng_throughput(dist, gen: int, calls: int, blocks: int, seed: int, sink,
                   stream=None) -> None:
    """sk_rng_throughput into a device uint32/int32 tensor of blocks * 256 words."""
    _check(lib().sk_rng_throughput(_dist(dist), gen, calls, blocks, seed, sink.data_ptr(),
                                   _stream(stream)), "sk_rng_throughput")


def sketch_rng_calls(ws, stream=None) -> int:
    """Generator calls of the last call-counting sketch on this workspace."""
    out = ctypes.c_uint64()
    _check(lib().sk_sketch_rng_calls(ws.data_ptr(), _stream(stream), ctypes.byref(out)),
           "sk_sketch_rng_calls")
    return int(out.value)


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


KERNEL_AUTO, KERNEL_TILE, KERNEL_KJI = 0, 1, 2


def plan_info(A: DeviceCsc, d: int, dist, prec: int = PREC_F32, tune=None) -> dict:
    """The cost model's view of a request (sk_plan_info)."""
    info = (ctypes.c_double * 6)()
    c = A.c_struct()
    _check(lib().sk_plan_info(ctypes.byref(c), d, _dist(dist), prec, _tuning(tune), info, 6),
           "sk_plan_info")
    return {"tile_us": info[0], "kji_us": info[1], "kernel": int(info[2]),
            "tile_cost": info[3], "variant": int(info[4]), "balance_sb": int(info[5])}


def autotune_measure(A: DeviceCsc, d: int, dist, seed: int, out, prec: int = PREC_F32,
                     ws=None, stream=None):
    """sk_autotune_measure: time the candidates on the device, cache the winner for
    the shape class; ``out`` (n, d) FP32 then holds the sketch with it.  Returns
    (tuning dict, ms)."""
    c = A.c_struct()
    if ws is None:
        need = ctypes.c_size_t()
        _check(lib().sk_autotune_workspace(ctypes.byref(c), d, _dist(dist), prec,
                                           ctypes.byref(need)), "sk_autotune_workspace")
        ws = alloc_workspace(int(need.value), out.device)
    t = SkTuning()
    ms = ctypes.c_double()
    _check(lib().sk_autotune_measure(ctypes.byref(c), d, _dist(dist), seed, prec,
                                     out.data_ptr(), d, ws.data_ptr(), ws.numel(),
                                     _stream(stream), ctypes.byref(t), ctypes.byref(ms)),
           "sk_autotune_measure")
    return tuning_dict(t), float(ms.value)


def plan_cache_lookup(A: DeviceCsc, d: int, dist, prec: int = PREC_F32):
    """The cached tuning of the request's shape class, or None."""
    t = SkTuning()
    c = A.c_struct()
    r = lib().sk_plan_cache_lookup(ctypes.byref(c), d, _dist(dist), prec, ctypes.byref(t))
    if r < 0 or r > 1:
        raise SketchError(r, "sk_plan_cache_lookup")
    return tuning_dict(t) if r == 1 else None


def plan_cache_clear() -> None:
    lib().sk_plan_cache_clear()


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


def qr_f64(A, stream=None):
    """Householder QR of a device FP64 tensor holding a d x n column-major matrix
    (torch shape (n, d)), in place; returns R as a torch (n, n) row-major view of
    the column-major R (i.e. R = returned.t())."""
    import torch
    n, d = A.shape
    need = ctypes.c_size_t()
    _check(lib().sk_qr_f64_workspace(d, n, ctypes.byref(need)), "sk_qr_f64_workspace")
    ws = alloc_workspace(need.value, A.device)
    R = torch.empty((n, n), dtype=torch.float64, device=A.device)
    _check(lib().sk_qr_f64(d, n, A.data_ptr(), d, R.data_ptr(), n, ws.data_ptr(), ws.numel(),
                           _stream(stream)), "sk_qr_f64")
    return R.t()


def trinv_f64(R, stream=None):
    """Inverse of an upper triangular FP64 matrix given as a torch (n, n) tensor
    (row-major); returns the inverse in the same convention."""
    import torch
    n = R.shape[0]
    Rc = R.t().contiguous()  # column-major storage
    out = torch.empty((n, n), dtype=torch.float64, device=R.device)
    _check(lib().sk_trinv_f64(n, Rc.data_ptr(), n, out.data_ptr(), n, _stream(stream)),
           "sk_trinv_f64")
    return out.t()


def svd_f64(M, stream=None):
    """One-sided Jacobi SVD of a tall FP64 matrix given as a torch (rows, n)
    tensor: returns (U diag(sigma) as (rows, n), V (n, n), sigma (n,), sweeps)
    with M = (U diag(sigma)) V^T; sigma in column order."""
    import torch
    rows, n = M.shape
    G = M.t().contiguous()  # column-major storage of M
    V = torch.empty((n, n), dtype=torch.float64, device=M.device)
    sig = torch.empty(n, dtype=torch.float64, device=M.device)
    need = ctypes.c_size_t()
    _check(lib().sk_svd_f64_workspace(rows, n, ctypes.byref(need)), "sk_svd_f64_workspace")
    ws = alloc_workspace(int(need.value), M.device)
    sweeps = ctypes.c_int32()
    _check(lib().sk_svd_f64(rows, n, G.data_ptr(), V.data_ptr(), sig.data_ptr(),
                            ctypes.byref(sweeps), ws.data_ptr(), ws.numel(), _stream(stream)),
           "sk_svd_f64")
    return G.t(), V.t(), sig, int(sweeps.value)


SAP_QR, SAP_SVD = 0, 1


def sap_params(d: int, dist, seed: int, atol: float = 1e-10, btol: float = 1e-10,
               conlim: float = 1e8, iter_lim: int = 1000, prec: int = PREC_F32,
               method: int = SAP_QR) -> SapParams:
    return SapParams(int(d), _dist(dist), int(prec), int(seed), float(atol), float(btol),
                     float(conlim), int(iter_lim), int(method))


class SapSolve:
    """One sketch-and-precondition least-squares solve on a device workspace.

    begin() enqueues sketch + QR + R^{-1} + LSQR start, iterate(k) enqueues k
    LSQR iterations, finish() enqueues x = R^{-1} y; all asynchronous on the
    given stream.  The solver info lives in the first bytes of the workspace."""

    INFO_BYTES = ctypes.sizeof(SapInfo)

    def __init__(self, A: DeviceCsc, b, params: SapParams, ws=None):
        import torch
        self.A = A
        self.c = A.c_struct()
        self.p = params
        self.b = b
        need = ctypes.c_size_t()
        _check(lib().sk_sap_workspace(ctypes.byref(self.c), ctypes.byref(self.p),
                                      ctypes.byref(need)), "sk_sap_workspace")
        self.ws_bytes = int(need.value)
        self.ws = ws if ws is not None else alloc_workspace(self.ws_bytes, A.colptr.device)
        self.x = torch.empty(A.n, dtype=torch.float64, device=A.colptr.device)

    @staticmethod
    def workspace_bytes(A: DeviceCsc, params: SapParams) -> int:
        need = ctypes.c_size_t()
        c = A.c_struct()
        _check(lib().sk_sap_workspace(ctypes.byref(c), ctypes.byref(params), ctypes.byref(need)),
               "sk_sap_workspace")
        return int(need.value)

    def begin(self, stream=None):
        _check(lib().sk_sap_begin(ctypes.byref(self.c), self.b.data_ptr(), ctypes.byref(self.p),
                                  self.ws.data_ptr(), self.ws_bytes, _stream(stream)),
               "sk_sap_begin")

    def iterate(self, iters: int, stream=None):
        _check(lib().sk_sap_iterate(ctypes.byref(self.c), ctypes.byref(self.p), int(iters),
                                    self.ws.data_ptr(), self.ws_bytes, _stream(stream)),
               "sk_sap_iterate")

    def finish(self, stream=None):
        _check(lib().sk_sap_finish(ctypes.byref(self.c), ctypes.byref(self.p), self.x.data_ptr(),
                                   self.ws.data_ptr(), self.ws_bytes, _stream(stream)),
               "sk_sap_finish")
        return self.x

    def info(self, stream=None) -> dict:
        """Synchronous read of the solver info (and the sketch's input status)."""
        inf = SapInfo()
        code = lib().sk_sap_read_info(ctypes.byref(self.c), ctypes.byref(self.p),
                                      self.ws.data_ptr(), self.ws_bytes, _stream(stream),
                                      ctypes.byref(inf))
        out = {f[0]: getattr(inf, f[0]) for f in SapInfo._fields_}
        out["status"] = int(code)
        return out

    @staticmethod
    def parse_info(raw: bytes) -> dict:
        inf = SapInfo.from_buffer_copy(raw[:ctypes.sizeof(SapInfo)])
        return {f[0]: getattr(inf, f[0]) for f in SapInfo._fields_}

    def solve(self, chunk: int = 16, stream=None) -> tuple:
        """Run to completion on one stream (polling between chunks)."""
        self.begin(stream)
        while True:
            self.iterate(chunk, stream)
            inf = self.info(stream)
            if inf["status"] != 0:
                raise SketchError(inf["status"], "sk_sap (sketch input)")
            if inf["done"]:
                break
        return self.finish(stream), inf


EXPORTED = ["sk_status_string", "sk_variant_count", "sk_sketch_workspace", "sk_sketch",
            "sk_sketch_status", "sk_materialize_s", "sk_rng_tables", "sk_autotune",
            "sk_sketch_batched_workspace", "sk_sketch_batched", "sk_sketch_batched_plan",
            "sk_sketch_batched_status", "sk_qr_f64_workspace", "sk_qr_f64", "sk_trinv_f64",
            "sk_sap_workspace", "sk_sap_begin", "sk_sap_iterate", "sk_sap_finish",
            "sk_sap_read_info", "sk_plan_info", "sk_autotune_workspace", "sk_autotune_measure",
            "sk_plan_cache_lookup", "sk_plan_cache_clear", "sk_svd_f64_workspace",
            "sk_svd_f64", "sk_sketch_colwise_f64"]
