"""Kernel choice and the measured autotuner (through the C-ABI).

The auto choice runs the Algorithm 3 loop-order kernel where the cost model
predicts it twice as fast as the S-tile kernel; the result is the same as
forcing that kernel (bit for bit) and within the element-wise bound of the
oracle.  The measured tuner leaves the sketch of its winner in A_hat, caches
the winner for the shape class, and sk_sketch with no tuning then runs it.
"""
import numpy as np
import pytest

from paper_2310_15419_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    from paper_2310_15419_amd import binding
    binding.lib()
    binding.plan_cache_clear()
    yield binding
    binding.plan_cache_clear()


def _sketch(B, dA, d, dist, seed, tune=None, prec=0):
    import torch
    ws = B.alloc_workspace(B.workspace_bytes(dA, d, dist, prec=prec, tune=tune))
    out = torch.full((dA.n, d), float("nan"), dtype=torch.float32, device="cuda")
    B.sketch_into(dA, d, dist, seed, out, ws, prec=prec, tune=tune)
    torch.cuda.synchronize()
    st = B.sketch_status(ws)
    assert st["status"] == 0, st
    return out


def _oracle_check(oracle_lib, out, A, d, dist, seed, what):
    got = out.t().cpu().numpy().astype(np.float64)
    ref = oracle_lib.sketch(A.m, A.n, A.colptr, A.rowidx, A.vals.astype(np.float64), d, dist,
                            seed)
    p = oracle_lib.parity(got, ref, A.colptr, A.vals, dist)
    print(f"{what}: {p}", flush=True)
    assert p["nonfinite"] == 0 and p["normwise"] <= 1e-5, p
    assert p["max_elem_scaled"] <= oracle_lib.ELEM_TOL, p


@pytest.mark.parametrize("shape,dist", [((20_000, 3000, 60_000, 900), "uniform"),
                                        ((10_000, 2000, 40_000, 6000), "rademacher")])
def test_auto_picks_colwise_and_matches(B, oracle_lib, shape, dist):
    import torch
    m, n, nnz, d = shape
    A = inputs.row_count_columns(m, n, nnz, 11)
    dA = B.DeviceCsc.from_host(A)
    assert B.plan_info(dA, d, dist)["kernel"] == B.KERNEL_KJI
    print(f"auto kernel {shape} {dist}", flush=True)
    auto = _sketch(B, dA, d, dist, 5)
    forced = _sketch(B, dA, d, dist, 5, tune={"kernel": B.KERNEL_KJI})
    assert torch.equal(auto, forced)
    _oracle_check(oracle_lib, auto, A, d, dist, 5, f"auto {dist}")
    tile = _sketch(B, dA, d, dist, 5, tune={"kernel": B.KERNEL_TILE})
    _oracle_check(oracle_lib, tile, A, d, dist, 5, f"tile {dist}")
    # the allocation-free form takes the same choice
    out = torch.full_like(auto, float("nan"))
    B.sketch_noalloc_into(dA, d, dist, 5, out)
    torch.cuda.synchronize()
    assert torch.equal(auto, out)


def test_measured_tuner_caches_its_winner(B, oracle_lib):
    import torch
    B.plan_cache_clear()
    A = inputs.uniform_positions(60_000, 700, 300_000, 3, "uniform", np.float32)
    dA = B.DeviceCsc.from_host(A)
    d = 1500
    assert B.plan_cache_lookup(dA, d, "gaussian") is None
    out = torch.full((A.n, d), float("nan"), dtype=torch.float32, device="cuda")
    print("measured tuner", flush=True)
    tune, ms = B.autotune_measure(dA, d, "gaussian", 9, out)
    torch.cuda.synchronize()
    print(f"winner {tune} {ms:.3f} ms", flush=True)
    assert ms > 0 and tune["kernel"] in (B.KERNEL_TILE, B.KERNEL_KJI)
    assert B.plan_cache_lookup(dA, d, "gaussian") == tune
    _oracle_check(oracle_lib, out, A, d, "gaussian", 9, "tuned")
    # the tuned A_hat is the explicit tuning's, and tune=None now runs it
    explicit = _sketch(B, dA, d, "gaussian", 9, tune=tune)
    assert torch.equal(out, explicit)
    assert torch.equal(_sketch(B, dA, d, "gaussian", 9), explicit)
    # another shape class is untouched; clearing the cache restores the model
    assert B.plan_cache_lookup(dA, 4 * d, "gaussian") is None
    B.plan_cache_clear()
    assert B.plan_cache_lookup(dA, d, "gaussian") is None


def test_measured_tuner_balance_stage(B, oracle_lib):
    # ten nonzeros per row over 1000 columns: the S-tile kernel wins, so the
    # third stage times the winner with the balanced row blocks switched;
    # the tuner's own workspace bound must hold both forms of every shape
    import torch
    B.plan_cache_clear()
    m, n, d = 300_000, 1000, 2000
    A = inputs.per_row_columns(m, n, 10, seed=31)
    dA = B.DeviceCsc.from_host(A)
    out = torch.full((n, d), float("nan"), dtype=torch.float32, device="cuda")
    print("measured tuner, balance stage", flush=True)
    tune, ms = B.autotune_measure(dA, d, "uniform", 17, out)
    torch.cuda.synchronize()
    print(f"winner {tune} {ms:.3f} ms", flush=True)
    assert tune["kernel"] == B.KERNEL_TILE and tune["balance"] in (0, 1, 2), tune
    explicit = _sketch(B, dA, d, "uniform", 17, tune=tune)
    assert torch.equal(out, explicit)
    sub = np.arange(0, n, 9)  # every ninth column against the oracle
    As = inputs.Csc(m, sub.size, np.concatenate([[0], np.cumsum(np.diff(A.colptr)[sub])]),
                    np.concatenate([A.rowidx[A.colptr[k]:A.colptr[k + 1]] for k in sub]),
                    np.concatenate([A.vals[A.colptr[k]:A.colptr[k + 1]] for k in sub]))
    _oracle_check(oracle_lib, out[sub], As, d, "uniform", 17, "tuned, column sample")
    B.plan_cache_clear()


def test_measured_tuner_precision_path(B, oracle_lib):
    import torch
    B.plan_cache_clear()
    # dense enough for the BF16 matrix-core path: only its splits are searched
    A = inputs.uniform_positions(20_000, 300, 120_000, 8, "uniform", np.float32)
    dA = B.DeviceCsc.from_host(A)
    d = 512
    out = torch.empty((A.n, d), dtype=torch.float32, device="cuda")
    tune, ms = B.autotune_measure(dA, d, "rademacher", 4, out, prec=B.PREC_BF16)
    torch.cuda.synchronize()
    assert tune["kernel"] == B.KERNEL_TILE and tune["variant"] == 0, tune
    ref = _sketch(B, dA, d, "rademacher", 4, tune=tune, prec=B.PREC_BF16)
    assert torch.equal(out, ref)
    B.plan_cache_clear()


def test_measured_tuner_reports_invalid_matrix(B):
    import torch
    A = inputs.uniform_positions(5000, 40, 3000, 2, "uniform", np.float32)
    r = A.rowidx.copy()
    r[4], r[5] = r[5], r[4]  # unsorted rows in a column
    if A.colptr[1] <= 5:
        pytest.skip("seeded matrix has a short first column")
    bad = B.DeviceCsc(A.m, A.n, torch.from_numpy(A.colptr).cuda(), torch.from_numpy(r).cuda(),
                      torch.from_numpy(A.vals).cuda())
    out = torch.empty((A.n, 64), dtype=torch.float32, device="cuda")
    with pytest.raises(B.SketchError) as e:
        B.autotune_measure(bad, 64, "uniform", 1, out)
    assert e.value.code == -2
    assert B.plan_cache_lookup(bad, 64, "uniform") is None
