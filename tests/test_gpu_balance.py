"""GPU parity of the balanced row blocks (sk_tuning.balance) against the FP64
oracle.

Rows dealt to blocks in a different order change only the summation order of
A_hat (S is a function of the row index), so the FP32 bar of the plain path
applies unchanged: normwise <= 1e-5, columns <= 1e-4, every element within
2^-20 of the scale of its terms.  Covered: the three distributions with many
super-blocks and a partial last one (kept in order), super-blocks holding
dense rows (kept in order), the value types of the renumbered copy, columns
with no entries in a super-block, bitwise reproducibility, the model's choice
on the plain-scale class, malformed input refused on the balanced path, and a
workspace's layout reused (phases 2|4|8) for other seeds and S rows.
"""
import numpy as np
import pytest

from paper_2310_15419_amd import inputs

pytestmark = pytest.mark.gpu

DISTS = ["rademacher", "uniform", "gaussian"]
TOL_NORM = 1e-5
TOL_COL = 1e-4


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    from paper_2310_15419_amd import binding
    binding.lib()
    return binding


def assert_parity(got, ref, A, dist, what=""):
    import oracle
    p = oracle.parity(got, ref, A.colptr, A.vals, dist)
    print(f"parity {what}: {p}", flush=True)
    assert p["nonfinite"] == 0, p
    assert p["normwise"] <= TOL_NORM and p["max_col"] <= TOL_COL, p
    assert p["max_elem_scaled"] <= oracle.ELEM_TOL, p
    return p


def run_gpu(B, A, d, dist, seed, tune=None, dtype=None, dA=None):
    dA = dA if dA is not None else B.DeviceCsc.from_host(A, dtype=dtype)
    out = B.sketch(dA, d, dist, seed, tune=tune)
    return out.cpu().numpy().astype(np.float64)


def run_oracle(oracle_lib, A, d, dist, seed):
    return oracle_lib.sketch(A.m, A.n, A.colptr, A.rowidx, A.vals.astype(np.float64), d, dist,
                             seed)


ON = {"kernel": 1, "balance": 2, "rows_per_block": 97}
OFF = {"kernel": 1, "balance": 1, "rows_per_block": 97}


@pytest.mark.parametrize("dist", DISTS)
def test_balanced_against_oracle(B, oracle_lib, dist):
    # 16 blocks of 97 rows per super-block: 38 full super-blocks and a partial
    # last one; 600 columns, six nonzeros per row (about one per (block, column))
    m, n, d = 60_000, 600, 150
    A = inputs.per_row_columns(m, n, 6, seed=11, dtype=np.float64)
    dA = B.DeviceCsc.from_host(A)
    assert B.plan_info(dA, d, dist, tune=ON)["balance_sb"] == 16
    assert B.plan_info(dA, d, dist, tune=OFF)["balance_sb"] == 0
    print(f"balanced {dist}", flush=True)
    ref = run_oracle(oracle_lib, A, d, dist, 7)
    got = run_gpu(B, A, d, dist, 7, tune=ON, dA=dA)
    assert_parity(got, ref, A, dist, "balanced")
    again = run_gpu(B, A, d, dist, 7, tune=ON, dA=dA)
    assert np.array_equal(got, again)  # bitwise reproducible
    assert_parity(run_gpu(B, A, d, dist, 7, tune=OFF, dA=dA), ref, A, dist, "in order")


def test_balanced_value_types(B, oracle_lib):
    import torch
    m, n, d = 30_000, 520, 64
    A = inputs.per_row_columns(m, n, 5, seed=12, dtype=np.float64)
    ref = run_oracle(oracle_lib, A, d, "uniform", 3)
    for dt in (np.float64, np.float32):
        print(f"balanced values {dt}", flush=True)
        assert_parity(run_gpu(B, A, d, "uniform", 3, tune=ON, dtype=dt), ref, A, "uniform", str(dt))
    vb = torch.from_numpy(A.vals).to(torch.bfloat16)
    Ab = inputs.Csc(A.m, A.n, A.colptr, A.rowidx, vb.to(torch.float64).numpy())
    dA = B.DeviceCsc(m, n, torch.from_numpy(A.colptr).cuda(), torch.from_numpy(A.rowidx).cuda(),
                     vb.cuda())
    print("balanced values bf16", flush=True)
    got = run_gpu(B, Ab, d, "uniform", 3, tune=ON, dA=dA)
    assert_parity(got, run_oracle(oracle_lib, Ab, d, "uniform", 3), Ab, "uniform", "bf16")


def test_balanced_with_dense_rows_and_empty_rows(B, oracle_lib):
    # power-law columns (some columns absent from most super-blocks), a block
    # of dense rows (their super-blocks stay in order, and the dense path
    # takes them), and many empty rows (positions are the nonempty rows)
    A, r0 = inputs.power_law_columns(200_000, 700, seed=13, max_frac=0.02, dense_rows=300,
                                     dtype=np.float64)
    d = 96
    for dist in ("gaussian", "rademacher"):
        print(f"balanced dense rows {dist}", flush=True)
        ref = run_oracle(oracle_lib, A, d, dist, 5)
        assert_parity(run_gpu(B, A, d, dist, 5, tune=ON), ref, A, dist, "balanced + dense")
        assert_parity(run_gpu(B, A, d, dist, 5, tune={"kernel": 1, "balance": 2}), ref, A, dist,
                      "balanced + dense, model rows")


def test_balanced_tiny_and_ragged(B, oracle_lib):
    # fewer rows than one super-block (kept in order) and a super-block of
    # exactly one block's worth of rows per block
    for m, n, rpb in ((500, 530, 31), (16 * 40, 515, 40), (16 * 40 + 1, 515, 40)):
        A = inputs.per_row_columns(m, n, 3, seed=m + n, dtype=np.float64)
        tune = {"kernel": 1, "balance": 2, "rows_per_block": rpb}
        for dist in DISTS:
            print(f"balanced tiny {m} {n} {rpb} {dist}", flush=True)
            ref = run_oracle(oracle_lib, A, 40, dist, 2)
            assert_parity(run_gpu(B, A, 40, dist, 2, tune=tune), ref, A, dist, f"tiny {m}")


def test_model_balances_plain_scale_class(B, oracle_lib):
    # the plain-scale class at a quarter of its rows (same columns, nonzeros
    # per row and d): the model takes balanced blocks; element-wise parity
    m, n, d = 500_000, 2000, 4000
    A = inputs.per_row_columns(m, n, 10, seed=20)
    dA = B.DeviceCsc.from_host(A)
    info = B.plan_info(dA, d, "uniform")
    assert info["kernel"] == 1 and info["balance_sb"] == 16, info
    print("plain-scale class, model plan", flush=True)
    got = run_gpu(B, A, d, "uniform", 21, dA=dA)
    sub = np.arange(0, n, 7)  # every seventh column against the oracle
    As = inputs.Csc(m, sub.size, np.concatenate([[0], np.cumsum(np.diff(A.colptr)[sub])]),
                    np.concatenate([A.rowidx[A.colptr[k]:A.colptr[k + 1]] for k in sub]),
                    np.concatenate([A.vals[A.colptr[k]:A.colptr[k + 1]] for k in sub]))
    ref = run_oracle(oracle_lib, As, d, "uniform", 21)
    assert_parity(got[:, sub], ref, As, "uniform", "plain-scale class")


def test_balanced_validation_errors(B):
    import torch
    m, n = 20_000, 600
    A = inputs.uniform_positions(m, n, 60_000, 3, "normal", np.float32)
    cases = {}
    r = A.rowidx.copy()
    lo = A.colptr[1]
    r[lo], r[lo + 1] = r[lo + 1], r[lo]
    cases["unsorted"] = (A.colptr, r, -2)
    r = A.rowidx.copy()
    r[7] = m
    cases["range"] = (A.colptr, r, -3)
    for name, (cp, ri, code) in cases.items():
        print(f"balanced validation {name}", flush=True)
        dA = B.DeviceCsc(m, n, torch.from_numpy(cp).cuda(), torch.from_numpy(ri).cuda(),
                         torch.from_numpy(A.vals).cuda())
        tune = {"kernel": 1, "balance": 2, "rows_per_block": 64}
        ws = B.alloc_workspace(B.workspace_bytes(dA, 40, "uniform", tune=tune))
        out = torch.zeros((n, 40), dtype=torch.float32, device="cuda")
        B.sketch_into(dA, 40, "uniform", 1, out, ws, tune=tune)
        st = B.sketch_status(ws)
        assert st["status"] == code, (name, st)
        assert torch.isnan(out).all().item()


def test_balanced_empty_matrix(B):
    import torch
    m, n = 50_000, 600
    dA = B.DeviceCsc(m, n, torch.zeros(n + 1, dtype=torch.int64, device="cuda"),
                     torch.zeros(0, dtype=torch.int32, device="cuda"),
                     torch.zeros(0, dtype=torch.float32, device="cuda"))
    print("balanced, no nonzeros", flush=True)
    out = B.sketch(dA, 64, "uniform", 1, tune={"kernel": 1, "balance": 2, "rows_per_block": 64})
    assert torch.equal(out, torch.zeros_like(out))


@pytest.mark.parametrize("balance", [1, 2])
def test_layout_reused_across_seeds_and_row_offsets(B, oracle_lib, balance):
    # a full call lays A out in the workspace; calls with phases 2|4|8 (S
    # tiles and accumulation, reduction, dense blocks) then sketch other
    # seeds and S-row offsets from that layout: bitwise equal to full calls,
    # and within the oracle's bar
    import torch
    m, n, d = 200_000, 1000, 512
    A = inputs.per_row_columns(m, n, 8, seed=41)
    dA = B.DeviceCsc.from_host(A)
    t = dict(B.autotune(dA, d, "uniform"), kernel=B.KERNEL_TILE, balance=balance)
    assert (B.plan_info(dA, d, "uniform", tune=t)["balance_sb"] > 0) == (balance == 2)
    ws = B.alloc_workspace(B.workspace_bytes(dA, d, "uniform", tune=t))
    out = torch.full((n, d), float("nan"), dtype=torch.float32, device="cuda")
    print(f"layout reuse, balance {balance}: full call", flush=True)
    B.sketch_into(dA, d, "uniform", 1, out, ws, tune=t)
    reuse = dict(t, phases=2 | 4 | 8)
    for seed, row0 in ((2, 0), (3, 777), (1, 5000)):
        print(f"layout reuse: seed {seed}, row0 {row0}", flush=True)
        got = torch.full((n, d), float("nan"), dtype=torch.float32, device="cuda")
        B.sketch_into(dA, d, "uniform", seed, got, ws, row0=row0, tune=reuse)
        full = torch.full((n, d), float("nan"), dtype=torch.float32, device="cuda")
        ws2 = B.alloc_workspace(B.workspace_bytes(dA, d, "uniform", tune=t))
        B.sketch_into(dA, d, "uniform", seed, full, ws2, row0=row0, tune=t)
        torch.cuda.synchronize()
        assert torch.equal(got, full), (seed, row0)
        del ws2
    sub = np.arange(0, n, 13)  # the last one against the oracle, a column sample
    As = inputs.Csc(m, sub.size, np.concatenate([[0], np.cumsum(np.diff(A.colptr)[sub])]),
                    np.concatenate([A.rowidx[A.colptr[k]:A.colptr[k + 1]] for k in sub]),
                    np.concatenate([A.vals[A.colptr[k]:A.colptr[k + 1]] for k in sub]))
    ref = oracle_lib.sketch(As.m, As.n, As.colptr, As.rowidx, As.vals.astype(np.float64), d,
                            "uniform", 1, row0=5000)
    assert_parity(got.cpu().numpy().astype(np.float64)[sub].T, ref, As, "uniform", "reused layout")
