"""Batched persistent launch: every item matches the oracle, and matches its
single-sketch call with the same tuning bitwise; per-item device validation."""
import numpy as np
import pytest

from paper_2310_15419_amd import inputs

pytestmark = pytest.mark.gpu
TOL_NORM, TOL_COL = 1e-5, 1e-4


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2310_15419_amd import binding
    binding.lib()
    return binding


def _items(seed, count, n_hi=500):
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        m = int(np.exp(rng.uniform(np.log(300), np.log(40_000))))
        n = int(rng.integers(1, n_hi + 1))
        d = int(rng.integers(2 * n, 4 * n + 1))
        rho = float(rng.uniform(0.005, 0.05))
        nnz = max(0, min(m * n, int(round(rho * m * n))))
        A = inputs.uniform_positions(m, n, nnz, int(rng.integers(1 << 30)), "uniform", np.float32)
        out.append((A, d, ["rademacher", "uniform", "gaussian"][b % 3], 5000 + b))
    return out


def _check(got, ref, A, dist, what):
    """The FP32 path's bar, element by element (see test_gpu_sketch)."""
    import oracle
    p = oracle.parity(got, ref, A.colptr, A.vals, dist)
    assert p["nonfinite"] == 0 and p["normwise"] <= TOL_NORM and p["max_col"] <= TOL_COL, (what, p)
    assert p["max_elem_scaled"] <= oracle.ELEM_TOL, (what, p)


def _rel(got, ref):
    diff = got - ref
    norm = np.linalg.norm(diff) / max(np.linalg.norm(ref), 1e-300)
    cref = np.linalg.norm(ref, axis=0)
    col = np.where(cref > 0, np.linalg.norm(diff, axis=0) / np.maximum(cref, 1e-300),
                   np.linalg.norm(diff, axis=0))
    return norm, (col.max() if col.size else 0.0)


def _run_batch(B, items, prec=0):
    import torch
    mats = [B.DeviceCsc.from_host(A) for A, _, _, _ in items]
    batch = B.Batch(mats, [d for _, d, _, _ in items], [s for _, _, s, _ in items],
                    [sd for _, _, _, sd in items], prec=prec)
    ws = B.alloc_workspace(batch.workspace_bytes())
    outs = [torch.full((A.n, d), float("nan"), dtype=torch.float32, device="cuda")
            for A, d, _, _ in items]
    batch.run(outs, ws)
    return batch, mats, outs, ws


@pytest.mark.parametrize("seed,n_hi", [(1, 500), (2, 64), (3, 1500)])
def test_batched_matches_oracle_and_single(B, oracle_lib, seed, n_hi):
    items = _items(seed, 18, n_hi)
    batch, mats, outs, ws = _run_batch(B, items)
    assert batch.status(ws) == [0] * len(items)
    plans = batch.plan()
    for i, ((A, d, dist, sd), dA, out, plan) in enumerate(zip(items, mats, outs, plans)):
        print(f"item {i}: m={A.m} n={A.n} nnz={A.nnz} d={d} {dist} plan={plan}", flush=True)
        got = out.t().cpu().numpy().astype(np.float64)
        ref = oracle_lib.sketch(A.m, A.n, A.colptr, A.rowidx, A.vals.astype(np.float64), d, dist,
                                sd)
        _check(got, ref, A, dist, i)
        single = B.sketch(dA, d, dist, sd, tune=plan).cpu().numpy().astype(np.float64)
        assert np.array_equal(single, got), i


def test_batched_edge_items_and_validation(B, oracle_lib):
    import torch
    items = _items(7, 6)
    # an empty matrix, a one-row matrix, and a matrix with unsorted rows
    E = inputs.Csc(500, 9, np.zeros(10, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32))
    one = inputs.uniform_positions(1, 5, 3, 1, "uniform", np.float32)
    bad = inputs.uniform_positions(800, 7, 300, 2, "uniform", np.float32)
    r = bad.rowidx.copy()
    lo = bad.colptr[3]
    r[lo], r[lo + 1] = r[lo + 1], r[lo]
    bad = inputs.Csc(bad.m, bad.n, bad.colptr, r, bad.vals)
    items += [(E, 20, "uniform", 1), (one, 12, "gaussian", 2), (bad, 16, "rademacher", 3)]
    batch, mats, outs, ws = _run_batch(B, items)
    st = batch.status(ws)
    assert st[:-1] == [0] * (len(items) - 1) and st[-1] == -2, st
    assert torch.count_nonzero(outs[-3]).item() == 0
    assert torch.isnan(outs[-1]).all().item()
    for (A, d, dist, sd), out in list(zip(items, outs))[:-1]:
        got = out.t().cpu().numpy().astype(np.float64)
        ref = oracle_lib.sketch(A.m, A.n, A.colptr, A.rowidx, A.vals.astype(np.float64), d, dist,
                                sd) if A.nnz else np.zeros((d, A.n))
        _check(got, ref, A, dist, (A.m, A.n, d))


@pytest.mark.parametrize("prec", [1, 2])  # BF16, FP8
def test_batched_precision_path(B, oracle_lib, prec):
    # +-1 items: the dense-enough ones on the matrix cores (within 1e-2 of
    # the FP64 oracle), the sparsest on the FP32 kernel (within 1e-5); each
    # bitwise equal to its single call with the reported tuning
    rng = np.random.default_rng(40 + prec)
    items = []
    for b in range(14):
        m = int(np.exp(rng.uniform(np.log(2_000), np.log(60_000))))
        n = int(rng.integers(20, 300))
        d = int(rng.integers(2 * n, 4 * n + 1))
        rho = 0.001 if b % 5 == 0 else float(rng.uniform(0.005, 0.08))
        A = inputs.uniform_positions(m, n, int(round(rho * m * n)), int(rng.integers(1 << 30)),
                                     "uniform", np.float32)
        items.append((A, d, "rademacher", 7000 + b))
    batch, mats, outs, ws = _run_batch(B, items, prec)
    assert batch.status(ws) == [0] * len(items)
    plans = batch.plan()
    for i, ((A, d, dist, sd), dA, out, plan) in enumerate(zip(items, mats, outs, plans)):
        mf = plan["variant"] == 0
        print(f"item {i}: m={A.m} n={A.n} nnz={A.nnz} d={d} mfma={mf}", flush=True)
        got = out.t().cpu().numpy().astype(np.float64)
        ref = oracle_lib.sketch(A.m, A.n, A.colptr, A.rowidx, A.vals.astype(np.float64), d, dist,
                                sd)
        norm, col = _rel(got, ref)
        assert norm <= (1e-2 if mf else TOL_NORM), (i, norm)
        assert mf == (A.nnz / (A.m * A.n) >= 0.01), i  # the batch's threshold
        single = B.sketch(dA, d, dist, sd, prec=prec, tune=plan).cpu().numpy().astype(np.float64)
        assert np.array_equal(single, got), i


def test_batched_many_small_items(B, oracle_lib):
    # 300 small items: workgroups of the item-indexed inspector kernels span
    # many items at once, and finding a workgroup's items takes more than
    # one step of the 32-way search
    rng = np.random.default_rng(11)
    items = []
    for b in range(300):
        m = int(rng.integers(50, 5000))
        n = int(rng.integers(1, 81))
        d = int(rng.integers(2 * n, 4 * n + 1))
        nnz = int(round(float(rng.uniform(0.0, 0.06)) * m * n))
        A = inputs.uniform_positions(m, n, nnz, int(rng.integers(1 << 30)), "uniform", np.float32)
        items.append((A, d, ["rademacher", "uniform", "gaussian"][b % 3], 7000 + b))
    batch, mats, outs, ws = _run_batch(B, items)
    assert batch.status(ws) == [0] * len(items)
    plans = batch.plan()
    check = set(int(i) for i in rng.choice(len(items), 12, replace=False))
    for i, ((A, d, dist, sd), dA, out, plan) in enumerate(zip(items, mats, outs, plans)):
        got = out.t().cpu().numpy().astype(np.float64)
        single = B.sketch(dA, d, dist, sd, tune=plan).cpu().numpy().astype(np.float64)
        assert np.array_equal(single, got), (i, A.m, A.n, A.nnz, d, dist)
        if i in check:
            ref = oracle_lib.sketch(A.m, A.n, A.colptr, A.rowidx, A.vals.astype(np.float64), d,
                                    dist, sd) if A.nnz else np.zeros((d, A.n))
            _check(got, ref, A, dist, i)
