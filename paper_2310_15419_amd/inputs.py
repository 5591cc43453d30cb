"""Seeded synthetic inputs (tall sparse CSC matrices) for the sketch S A.

Holds no part of the sketch's arithmetic: numpy's generator only.  Used by
both the tests (oracle side and HIP side) and the benchmark.  The workload
shapes stand in for the paper's matrices (Tables I and VIII), which are not
available; see the design notes for each recipe.

A CSC matrix is returned as ``Csc(m, n, colptr int64[n+1], rowidx int32[nnz],
vals float[nnz])`` with row indices sorted and unique within each column.
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np


@dataclasses.dataclass
class Csc:
    m: int
    n: int
    colptr: np.ndarray
    rowidx: np.ndarray
    vals: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.rowidx.size)

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csc_matrix((self.vals, self.rowidx, self.colptr), shape=(self.m, self.n))

    def to_dense(self) -> np.ndarray:
        out = np.zeros((self.m, self.n), dtype=np.float64)
        for k in range(self.n):
            lo, hi = self.colptr[k], self.colptr[k + 1]
            out[self.rowidx[lo:hi], k] = self.vals[lo:hi]
        return out

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in (self.colptr, self.rowidx, self.vals):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()

    def astype(self, dtype) -> "Csc":
        return Csc(self.m, self.n, self.colptr, self.rowidx, self.vals.astype(dtype))


def from_coo(m: int, n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray) -> Csc:
    """CSC from unique (row, col) pairs (sorted by column, then row)."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    key = cols * np.int64(m) + rows
    order = np.argsort(key, kind="stable")
    key = key[order]
    if key.size > 1 and np.any(key[1:] == key[:-1]):
        raise ValueError("duplicate (row, col) positions")
    counts = np.bincount(cols, minlength=n)
    colptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=colptr[1:])
    return Csc(m, n, colptr, rows[order].astype(np.int32), np.asarray(vals)[order])


def uniform_positions(m: int, n: int, nnz: int, seed: int, dist: str = "normal",
                      dtype=np.float64) -> Csc:
    """``nnz`` distinct positions drawn uniformly without replacement from m*n."""
    rng = np.random.default_rng(seed)
    total = m * n
    if nnz > total:
        raise ValueError("nnz > m*n")
    if nnz * 4 > total:
        flat = rng.choice(total, size=nnz, replace=False)
    else:
        flat = np.unique(rng.integers(0, total, size=int(nnz * 1.2) + 16))
        while flat.size < nnz:
            flat = np.unique(np.concatenate([flat, rng.integers(0, total, size=nnz)]))
        flat = rng.permutation(flat)[:nnz]
    rows, cols = flat % m, flat // m
    vals = _values(rng, nnz, dist, dtype)
    return from_coo(m, n, rows, cols, vals)


def _values(rng, size, dist, dtype):
    if dist == "normal":
        v = rng.standard_normal(size)
    elif dist == "uniform":
        v = rng.uniform(-1.0, 1.0, size)
    elif dist == "ones":
        v = np.ones(size)
    else:
        raise ValueError(dist)
    return v.astype(dtype)


def per_row_columns(m: int, n: int, per_row: int, seed: int, dtype=np.float32,
                    chunk: int = 1 << 20) -> Csc:
    """Every row holds exactly ``per_row`` distinct uniformly random columns;
    values U(-1, 1)."""
    rng = np.random.default_rng(seed)
    cols = np.empty((m, per_row), dtype=np.int32)
    for r0 in range(0, m, chunk):
        r1 = min(m, r0 + chunk)
        c = rng.integers(0, n, size=(r1 - r0, per_row), dtype=np.int32)
        while True:
            cs = np.sort(c, axis=1)
            bad = np.any(cs[:, 1:] == cs[:, :-1], axis=1)
            if not bad.any():
                break
            c[bad] = rng.integers(0, n, size=(int(bad.sum()), per_row), dtype=np.int32)
        cols[r0:r1] = c
    rows = np.repeat(np.arange(m, dtype=np.int64), per_row)
    cols = cols.reshape(-1).astype(np.int64)
    vals = rng.uniform(-1.0, 1.0, rows.size).astype(dtype)
    return from_coo(m, n, rows, cols, vals)


def power_law_columns(m: int, n: int, seed: int, max_frac: float = 0.05, dense_rows: int = 0,
                      dtype=np.float32) -> tuple[Csc, int]:
    """Column nnz by rank r = 1..n: c_r = max(1, floor(max_frac*m / r^2)), placed over a
    seeded column permutation, rows uniform without replacement; plus (optionally) a dense
    block of ``dense_rows`` consecutive rows at a random offset (dense wins on overlap).
    Values U(-1, 1).  Returns (A, dense_row_offset)."""
    rng = np.random.default_rng(seed)
    ranks = np.arange(1, n + 1, dtype=np.float64)
    counts = np.maximum(1, np.floor(max_frac * m / ranks ** 2)).astype(np.int64)
    perm = rng.permutation(n)
    rows_l, cols_l = [], []
    for r_i in range(n):
        c = int(counts[r_i])
        k = int(perm[r_i])
        rows_l.append(rng.choice(m, size=c, replace=False) if c * 4 > m
                      else _distinct_ints(rng, m, c))
        cols_l.append(np.full(c, k, dtype=np.int64))
    rows = np.concatenate(rows_l).astype(np.int64)
    cols = np.concatenate(cols_l)
    r0 = -1
    if dense_rows > 0:
        r0 = int(rng.integers(0, m - dense_rows + 1))
        keep = (rows < r0) | (rows >= r0 + dense_rows)
        rows, cols = rows[keep], cols[keep]
        dr = np.repeat(np.arange(r0, r0 + dense_rows, dtype=np.int64), n)
        dc = np.tile(np.arange(n, dtype=np.int64), dense_rows)
        rows = np.concatenate([rows, dr])
        cols = np.concatenate([cols, dc])
    vals = rng.uniform(-1.0, 1.0, rows.size).astype(dtype)
    return from_coo(m, n, rows, cols, vals), r0


def _distinct_ints(rng, hi: int, count: int) -> np.ndarray:
    out = np.unique(rng.integers(0, hi, size=count + 8))
    while out.size < count:
        out = np.unique(np.concatenate([out, rng.integers(0, hi, size=count)]))
    return rng.permutation(out)[:count]


# ------------------------------------------------------------ workloads
def workload_plain_small(seed: int = 0) -> Csc:
    """m=1e5, n=200, 2e5 distinct uniform positions (1% density), values N(0,1), FP64."""
    return uniform_positions(100_000, 200, 200_000, seed, "normal", np.float64)


def workload_plain_scale(seed: int = 20, m: int = 2_000_000, n: int = 2000, per_row: int = 10) -> Csc:
    """m=2e6, n=2000, 10 distinct uniform columns per row (nnz=2e7), values U(-1,1), FP32."""
    return per_row_columns(m, n, per_row, seed, np.float32)


def workload_skewed(seed: int = 30, m: int = 4_000_000, n: int = 1000, dense_rows: int = 2000):
    """m=4e6, n=1000, power-law column nnz (exponent 2, max 5% of m) plus a dense
    2000-row block at a random offset; values U(-1,1), FP32."""
    return power_law_columns(m, n, seed, 0.05, dense_rows, np.float32)


# ------------------------------------------- the paper's SpMM test shapes
# (m, n, nnz) of the matrices of Table I (SuiteSparse; the sketch has d = 3n
# rows there).  The matrices themselves are not available: the stand-ins keep
# the shape, the nonzero count and the nonzeros per row (3, 4, 3, 3.65 and 5),
# with the columns uniform at random.
TABLE1 = {
    "mk-12": (13860, 1485, 41580),
    "ch7-9-b3": (105840, 17640, 423360),
    "shar_te2-b2": (200200, 17160, 600600),
    "mesh_deform": (234023, 9393, 853829),
    "cis-n4c6-b4": (20058, 5970, 100290),
}


def row_count_columns(m: int, n: int, nnz: int, seed: int, dtype=np.float32) -> Csc:
    """nnz nonzeros spread over the rows as evenly as possible (floor or ceil
    of nnz/m per row, the extra ones on random rows), distinct uniformly random
    columns in each row; values U(-1,1)."""
    rng = np.random.default_rng(seed)
    base = nnz // m
    extra = np.zeros(m, dtype=bool)
    extra[rng.choice(m, size=nnz - base * m, replace=False)] = True
    k = base + 1
    cols = rng.integers(0, n, size=(m, k), dtype=np.int64)
    while True:
        cs = np.sort(cols, axis=1)
        bad = np.any(cs[:, 1:] == cs[:, :-1], axis=1)
        if not bad.any():
            break
        cols[bad] = rng.integers(0, n, size=(int(bad.sum()), k), dtype=np.int64)
    keep = np.ones((m, k), dtype=bool)
    keep[~extra, k - 1] = False
    rows = np.repeat(np.arange(m, dtype=np.int64), k).reshape(m, k)[keep]
    cols = cols[keep]
    vals = rng.uniform(-1.0, 1.0, rows.size).astype(dtype)
    return from_coo(m, n, rows, cols, vals)


def table1_standin(name: str, seed: int = 60) -> tuple[Csc, int]:
    """The stand-in for a Table I matrix and its sketch size d = 3n."""
    m, n, nnz = TABLE1[name]
    return row_count_columns(m, n, nnz, seed), 3 * n


def abnormal(kind: str, m: int = 100_000, n: int = 10_000, seed: int = 70,
             dtype=np.float32) -> Csc:
    """The exotic sparsity patterns of Table VI (density about 1e-3):
    A -- every 1000th row dense, all other rows empty;
    B -- about 2998/3000 of the nonzeros in the middle third of the columns
         (uniform there), the rest uniform over the other columns;
    C -- every 1000th column dense, all other columns empty.
    Values U(-1,1)."""
    rng = np.random.default_rng(seed)
    step = 1000
    if kind == "A":
        r = np.arange(0, m, step, dtype=np.int64)
        rows = np.repeat(r, n)
        cols = np.tile(np.arange(n, dtype=np.int64), r.size)
    elif kind == "C":
        c = np.arange(0, n, step, dtype=np.int64)
        rows = np.tile(np.arange(m, dtype=np.int64), c.size)
        cols = np.repeat(c, m)
    elif kind == "B":
        nnz = int(round(1e-3 * m * n))
        mid = int(round(nnz * 2998 / 3000))
        c0, c1 = n // 3, 2 * n // 3
        inside = c0 * m + _distinct_ints(rng, (c1 - c0) * m, mid)
        outside_n = n - (c1 - c0)
        o = _distinct_ints(rng, outside_n * m, nnz - mid)
        oc = o // m
        oc = np.where(oc < c0, oc, oc + (c1 - c0))  # skip the middle block
        flat = np.concatenate([inside, oc * m + o % m])
        rows, cols = flat % m, flat // m
    else:
        raise ValueError(kind)
    vals = rng.uniform(-1.0, 1.0, rows.size).astype(dtype)
    return from_coo(m, n, rows, cols, vals)


@dataclasses.dataclass
class BatchItem:
    A: Csc
    d: int
    seed: int
    density: float


def workload_batched_specs(count: int = 512, seed: int = 40, m_lo: int = 10_000,
                           m_hi: int = 500_000, n_lo: int = 50, n_hi: int = 500,
                           rho_lo: float = 0.005, rho_hi: float = 0.05) -> list[tuple]:
    """The items' shapes: (m, n, d, nnz, matrix seed, S seed, rho) per item, drawn in
    order from one seeded stream (m log-uniform, n and d uniform, d in [2n, 4n])."""
    rng = np.random.default_rng(seed)
    specs = []
    for b in range(count):
        m = int(np.floor(np.exp(rng.uniform(np.log(m_lo), np.log(m_hi)))))
        n = int(rng.integers(n_lo, n_hi + 1))
        d = int(rng.integers(2 * n, 4 * n + 1))
        rho = float(rng.uniform(rho_lo, rho_hi))
        nnz = int(round(rho * m * n))
        specs.append((m, n, d, nnz, int(rng.integers(0, 2**31)), 40000 + b, rho))
    return specs


def _batched_item(spec) -> BatchItem:
    m, n, d, nnz, mseed, sseed, rho = spec
    return BatchItem(uniform_positions(m, n, nnz, mseed, "uniform", np.float32), d, sseed, rho)


def workload_batched(count: int = 512, seed: int = 40, workers: int = 1, **kw) -> list[BatchItem]:
    """``count`` independent sketches: m log-uniform, n uniform, d uniform in [2n, 4n],
    density uniform, exact round(rho m n) positions, values U(-1,1) FP32; S seed 40000+b.
    ``workers`` > 1 generates the items in a process pool (same items)."""
    specs = workload_batched_specs(count, seed, **kw)
    if workers <= 1:
        return [_batched_item(s) for s in specs]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_batched_item, specs, chunksize=1)


def ls_request(seed: int, m: int, n: int, dense_rows: int = 2000, noise: float = 1e-6,
               max_frac: float = 0.05):
    """A least-squares request min ||Ax - b||: A from the power-law generator with a dense
    block of max(dense_rows, n) rows (full column rank), x_true ~ N(0, I),
    b = A x_true + noise * N(0, I).  Returns (A FP64, b, x_true)."""
    A, _ = power_law_columns(m, n, seed, max_frac, max(dense_rows, n), np.float64)
    rng = np.random.default_rng(seed + 7919)
    x = rng.standard_normal(n)
    b = A.to_scipy() @ x + noise * rng.standard_normal(m)
    return A, b, x


def ls_request_rank_deficient(seed: int, m: int, n: int, rank: int, dense_rows: int = 300,
                              near: float = 0.0, noise: float = 1e-6):
    """A least-squares request whose A has singular values at or near zero (the
    role of the numerically rank-deficient matrices of Sec. V-E-1): `rank`
    base columns from the power-law generator with a dense block, values on
    the grid k/1024 (so sums of them are exact in FP32 and FP64); then n - rank
    dependent columns, in turn an exact sum of two base columns, a power-of-two
    multiple of one, and an empty column.  near > 0 adds to the first
    dependent column one entry of that size in a row where it has none (the
    column is then independent, with a singular value of about `near`).
    x_true ~ N(0, I), b = A x_true + noise * N(0, I).

    Returns (A FP64, b, null) with null the list of dependencies: (j, {col:
    coefficient}) meaning column j = sum coefficient * column, exact (the
    first one not exact when near > 0)."""
    if not 2 <= rank < n:
        raise ValueError("need 2 <= rank < n")
    base, _ = power_law_columns(m, rank, seed, 0.05, max(dense_rows, rank), np.float64)
    q = np.round(base.vals * 1024.0)
    q[q == 0] = 1.0
    rng = np.random.default_rng(seed + 104729)
    cols = {}
    for k in range(rank):
        sl = slice(base.colptr[k], base.colptr[k + 1])
        cols[k] = dict(zip(base.rowidx[sl].tolist(), (q[sl] / 1024.0).tolist()))
    null = []
    for j in range(rank, n):
        kind = (j - rank) % 3
        if kind == 0:
            a, c = (int(v) for v in rng.choice(rank, size=2, replace=False))
            col = dict(cols[a])
            for r_, v in cols[c].items():
                col[r_] = col.get(r_, 0.0) + v
            null.append((j, {a: 1.0, c: 1.0}))
        elif kind == 1:
            a = int(rng.integers(rank))
            f = float(2.0 ** int(rng.integers(-3, 4)))
            col = {r_: f * v for r_, v in cols[a].items()}
            null.append((j, {a: f}))
        else:
            col = {}
            null.append((j, {}))
        cols[j] = col
    if near > 0.0:
        j0 = rank
        free = np.setdiff1d(np.arange(m), np.fromiter(cols[j0].keys(), dtype=np.int64))
        cols[j0][int(rng.choice(free))] = near
    rows, cidx, vals = [], [], []
    for j in range(n):
        items = sorted(cols[j].items())
        rows.extend(r_ for r_, _ in items)
        cidx.extend([j] * len(items))
        vals.extend(v for _, v in items)
    A = from_coo(m, n, np.array(rows, dtype=np.int64), np.array(cidx, dtype=np.int64),
                 np.array(vals, dtype=np.float64))
    x = rng.standard_normal(n)
    b = A.to_scipy() @ x + noise * rng.standard_normal(m)
    return A, b, null
