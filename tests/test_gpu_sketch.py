"""GPU parity of the HIP sketch against the FP64 oracle (through the C-ABI).

Bar: S bit-exact; on the FP32 path A_hat's normwise relative error <= 1e-5,
each column within 1e-4, and every element within 2^-20 of the scale of the
terms summed into it (max|S| sum_j |a_jk|); identity blocks bit-exact;
results bitwise reproducible for a fixed tuning.
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


def rel_errors(got, ref):
    got = np.asarray(got, dtype=np.float64)
    diff = got - ref
    norm = np.linalg.norm(diff) / max(np.linalg.norm(ref), 1e-300)
    colref = np.linalg.norm(ref, axis=0)
    col = np.linalg.norm(diff, axis=0) / np.maximum(colref, 1e-300)
    col = np.where(colref > 0, col, np.linalg.norm(diff, axis=0))
    return norm, float(col.max()) if col.size else 0.0


def assert_parity(got, ref, A, dist, what=""):
    """The FP32 path's bar: normwise and per-column relative errors, and every
    element within ELEM_TOL of the scale of the terms summed into it."""
    import oracle
    p = oracle.parity(got, ref, A.colptr, A.vals, dist)
    print(f"parity {what}: {p}", flush=True)
    assert p["nonfinite"] == 0, p
    assert p["normwise"] <= TOL_NORM and p["max_col"] <= TOL_COL, p
    assert p["max_elem_scaled"] <= oracle.ELEM_TOL, p
    return p


def run_gpu(B, A, d, dist, seed, row0=0, tune=None, dtype=None):
    dA = B.DeviceCsc.from_host(A, dtype=dtype)
    out = B.sketch(dA, d, dist, seed, row0=row0, tune=tune)
    return out.cpu().numpy().astype(np.float64)


def run_oracle(oracle_lib, A, d, dist, seed, row0=0):
    return oracle_lib.sketch(A.m, A.n, A.colptr, A.rowidx, A.vals.astype(np.float64), d, dist,
                             seed, row0=row0)


# ------------------------------------------------------------------ S
@pytest.mark.parametrize("dist", DISTS)
@pytest.mark.parametrize("row0,d,col0,ncols", [(0, 256, 0, 300), (3, 131, 99_990, 17),
                                               (126, 70, 2**31 - 5, 4), (1, 9, 2**40 + 3, 5)])
def test_materialize_bit_exact(B, oracle_lib, dist, row0, d, col0, ncols):
    print(f"materialize {dist} row0={row0} d={d} col0={col0}", flush=True)
    got = B.materialize_s(row0, d, col0, ncols, dist, 1234).cpu().numpy().astype(np.float64)
    ref = oracle_lib.materialize_s(dist, 1234, row0, d, col0, ncols)
    assert np.array_equal(got, ref)


# ------------------------------------------------------------- A_hat
@pytest.mark.parametrize("dist", DISTS)
@pytest.mark.parametrize("variant", list(range(0, 11)))
def test_sketch_small_all_variants(B, oracle_lib, dist, variant):
    # several tiles in d, several row blocks, ragged tails everywhere
    m, n, d = 7001, 77, 203
    A = inputs.uniform_positions(m, n, 9000, 5, "normal", np.float64)
    tune = {"variant": variant, "rows_per_block": 97} if variant else None
    print(f"sketch small {dist} variant={variant}", flush=True)
    got = run_gpu(B, A, d, dist, 42, tune=tune)
    ref = run_oracle(oracle_lib, A, d, dist, 42)
    assert_parity(got, ref, A, dist, f"variant {variant}")


# ------------------------------------------- the benchmarked shapes
def test_plain_small_workload_full_size(B, oracle_lib):
    # the plain small workload exactly: m = 1e5, n = 200, 2e5 uniform
    # positions, FP64 N(0,1) values, +-1 S (seed 1), d = 400
    A = inputs.workload_plain_small()
    print("plain small workload, full size", flush=True)
    got = run_gpu(B, A, 400, "rademacher", 1)
    ref = run_oracle(oracle_lib, A, 400, "rademacher", 1)
    assert_parity(got, ref, A, "rademacher", "plain small")


def test_skewed_workload_class(B, oracle_lib):
    # the skewed generator at a tenth of its rows (m = 4e5): power-law
    # columns, a dense 2000-row block (the matrix-core path), heavy-column
    # folding, Gaussian S at d = 3000 (94 S-row tiles)
    A, r0 = inputs.power_law_columns(400_000, 1000, 30, 0.05, 2000, np.float32)
    print(f"skewed class m=4e5 (dense block at row {r0})", flush=True)
    got = run_gpu(B, A, 3000, "gaussian", 31)
    ref = run_oracle(oracle_lib, A, 3000, "gaussian", 31)
    assert_parity(got, ref, A, "gaussian", "skewed class")


def test_plain_scale_workload_class(B, oracle_lib):
    # the plain-at-scale generator at a tenth of its rows (m = 2e5, n = 2000,
    # 10 columns per row), uniform S at d = 4000
    A = inputs.per_row_columns(200_000, 2000, 10, 20)
    print("plain scale class m=2e5", flush=True)
    got = run_gpu(B, A, 4000, "uniform", 21)
    ref = run_oracle(oracle_lib, A, 4000, "uniform", 21)
    assert_parity(got, ref, A, "uniform", "plain scale class")


@pytest.mark.parametrize("dist", DISTS)
def test_tiling_independence(B, oracle_lib, dist):
    m, n, d = 20_000, 150, 300
    A = inputs.uniform_positions(m, n, 30_000, 8, "uniform", np.float32)
    ref = run_oracle(oracle_lib, A, d, dist, 3)
    outs = []
    for tune in [None, {"rows_per_block": 64, "splits": 3}, {"rows_per_block": 1000, "splits": 1},
                 {"variant": 6, "splits": 16}, {"variant": 5, "rows_per_block": 31},
                 {"variant": 1, "row_pad": 4}, {"variant": 3, "row_pad": 8, "tile_rows": 64}]:
        print(f"tiling {dist} {tune}", flush=True)
        got = run_gpu(B, A, d, dist, 3, tune=tune)
        assert_parity(got, ref, A, dist, str(tune))
        outs.append(got)


@pytest.mark.parametrize("dist", DISTS)
def test_identity_blocks_exact(B, oracle_lib, dist):
    m, n, d = 50_000, 300, 257
    rng = np.random.default_rng(2)
    p = rng.choice(m, size=n, replace=False)
    e = rng.integers(-3, 4, size=n)
    A = inputs.from_coo(m, n, p, np.arange(n), (2.0 ** e).astype(np.float32))
    got = run_gpu(B, A, d, dist, 11)
    S = np.stack([oracle_lib.materialize_s(dist, 11, 0, d, int(pk), 1)[:, 0] for pk in p], axis=1)
    assert np.array_equal(got, S * (2.0 ** e)[None, :])


def test_row0_stacking_and_determinism(B, oracle_lib):
    m, n, d = 30_000, 64, 200
    A = inputs.uniform_positions(m, n, 40_000, 13, "uniform", np.float32)
    for dist in DISTS:
        full = run_gpu(B, A, d, dist, 5)
        again = run_gpu(B, A, d, dist, 5)
        assert np.array_equal(full, again)  # bitwise reproducible
        top = run_gpu(B, A, 70, dist, 5)
        bot = run_gpu(B, A, d - 70, dist, 5, row0=70)
        ref = run_oracle(oracle_lib, A, d - 70, dist, 5, row0=70)
        assert_parity(bot, ref, A, dist, "row0 = 70")
        assert_parity(np.concatenate([top, bot]), full, A, dist, "stacked")


def test_value_types(B, oracle_lib):
    import torch
    m, n, d = 9000, 40, 96
    A = inputs.uniform_positions(m, n, 12_000, 21, "uniform", np.float64)
    ref = run_oracle(oracle_lib, A, d, "uniform", 9)
    for dt in (np.float64, np.float32):
        assert_parity(run_gpu(B, A, d, "uniform", 9, dtype=dt), ref, A, "uniform", str(dt))
    # bf16 values: compare with the oracle on the bf16-rounded values
    vb = torch.from_numpy(A.vals).to(torch.bfloat16)
    Ab = inputs.Csc(A.m, A.n, A.colptr, A.rowidx, vb.to(torch.float64).numpy())
    dA = B.DeviceCsc(m, n, torch.from_numpy(A.colptr).cuda(), torch.from_numpy(A.rowidx).cuda(),
                     vb.cuda())
    got = B.sketch(dA, d, "uniform", 9).cpu().numpy().astype(np.float64)
    assert_parity(got, run_oracle(oracle_lib, Ab, d, "uniform", 9), Ab, "uniform", "bf16")


def test_edge_shapes(B, oracle_lib):
    cases = [(1, 1, 1, 1), (5, 3, 1, 2), (1000, 1, 1, 1000), (64, 64, 4096, 5), (300, 2, 600, 9)]
    for m, n, nnz, d in cases:
        nnz = min(nnz, m * n)
        A = inputs.uniform_positions(m, n, nnz, m + n, "normal", np.float64)
        for dist in DISTS:
            print(f"edge {m} {n} {nnz} {d} {dist}", flush=True)
            got = run_gpu(B, A, d, dist, 1)
            ref = run_oracle(oracle_lib, A, d, dist, 1)
            assert_parity(got, ref, A, dist, f"edge {m} {n} {nnz} {d}")


def test_empty_matrix_gives_zeros(B):
    import torch
    m, n, d = 1000, 7, 33
    dA = B.DeviceCsc(m, n, torch.zeros(n + 1, dtype=torch.int64, device="cuda"),
                     torch.zeros(0, dtype=torch.int32, device="cuda"),
                     torch.zeros(0, dtype=torch.float32, device="cuda"))
    out = B.sketch(dA, d, "gaussian", 1)
    assert torch.count_nonzero(out).item() == 0


def test_device_validation_errors(B):
    import torch
    m, n = 500, 6
    A = inputs.uniform_positions(m, n, 400, 3, "normal", np.float32)
    cases = {}
    r = A.rowidx.copy()
    lo = A.colptr[1]
    r[lo], r[lo + 1] = r[lo + 1], r[lo]
    cases["unsorted"] = (A.colptr, r, -2)
    r = A.rowidx.copy()
    r[7] = m
    cases["range"] = (A.colptr, r, -3)
    cp = A.colptr.copy()
    cp[n] = cp[n] - 1
    cases["colptr"] = (cp, A.rowidx, -7)
    for name, (cp, ri, code) in cases.items():
        print(f"validation {name}", flush=True)
        dA = B.DeviceCsc(m, n, torch.from_numpy(cp).cuda(), torch.from_numpy(ri).cuda(),
                         torch.from_numpy(A.vals).cuda())
        ws = B.alloc_workspace(B.workspace_bytes(dA, 40, "uniform"))
        out = torch.zeros((n, 40), dtype=torch.float32, device="cuda")
        B.sketch_into(dA, 40, "uniform", 1, out, ws)
        st = B.sketch_status(ws)
        assert st["status"] == code, (name, st)
        assert torch.isnan(out).all().item()
        with pytest.raises(B.SketchError):
            B.sketch(dA, 40, "uniform", 1)


def test_nonempty_row_count(B):
    import torch
    m, n = 100_000, 200
    A = inputs.workload_plain_small(seed=0)
    dA = B.DeviceCsc.from_host(A)
    ws = B.alloc_workspace(B.workspace_bytes(dA, 8, "rademacher"))
    out = torch.empty((n, 8), dtype=torch.float32, device="cuda")
    B.sketch_into(dA, 8, "rademacher", 1, out, ws)
    st = B.sketch_status(ws)
    assert st["status"] == 0
    assert st["nonempty_rows"] == np.unique(A.rowidx).size
    assert abs(st["nonempty_rows"] - m * (1 - (1 - 0.01) ** n)) < 5 * np.sqrt(m * 0.25)


@pytest.mark.parametrize("dist", DISTS)
def test_multi_pass_blocks(B, oracle_lib, dist):
    # dense rows: a block's entries exceed one LDS staging pass
    m, n, d = 3000, 256, 100
    A = inputs.uniform_positions(m, n, int(0.3 * m * n), 77, "uniform", np.float32)
    ref = run_oracle(oracle_lib, A, d, dist, 6)
    for tune in [{"variant": 5, "rows_per_block": 1500}, {"variant": 1, "rows_per_block": 2000},
                 None]:
        print(f"multi-pass {dist} {tune}", flush=True)
        got = run_gpu(B, A, d, dist, 6, tune=tune)
        assert_parity(got, ref, A, dist, str(tune))


@pytest.mark.parametrize("dist", DISTS)
def test_dense_blocks_mfma(B, oracle_lib, dist):
    # power-law columns plus a dense row block: blocks above the density
    # threshold run on the matrix cores; every threshold gives the same A_hat
    A, r0 = inputs.power_law_columns(60_000, 130, 31, 0.05, 700, np.float32)
    d = 270
    ref = run_oracle(oracle_lib, A, d, dist, 8)
    for tune in [None, {"dense_min_pct": 101}, {"dense_min_pct": 5},
                 {"dense_min_pct": 40, "rows_per_block": 300, "splits": 3}]:
        print(f"dense {dist} {tune}", flush=True)
        got = run_gpu(B, A, d, dist, 8, tune=tune)
        assert_parity(got, ref, A, dist, str(tune))
    # misaligned S-row offset on the dense path
    got = run_gpu(B, A, 130, dist, 8, row0=3, tune={"dense_min_pct": 5})
    assert_parity(got, run_oracle(oracle_lib, A, 130, dist, 8, row0=3), A, dist, "row0 = 3")


@pytest.mark.parametrize("dist", DISTS)
def test_heavy_column_split(B, oracle_lib, dist):
    # power-law columns: the heaviest columns are split into interleaved
    # virtual columns and summed back in fixed order; forced on, forced off
    # and with the other tiling knobs, the result matches the oracle
    A, _ = inputs.power_law_columns(60_000, 130, 41, 0.2, 0, np.float32)
    d = 190
    ref = run_oracle(oracle_lib, A, d, dist, 4)
    outs = {}
    for tune in [{"col_split": 1}, {"col_split": 2}, {"col_split": 2, "dense_min_pct": 101},
                 {"col_split": 2, "variant": 1, "rows_per_block": 300, "splits": 3},
                 {"col_split": 2, "variant": 6, "dense_min_pct": 5}]:
        print(f"col split {dist} {tune}", flush=True)
        got = run_gpu(B, A, d, dist, 4, tune=tune)
        assert_parity(got, ref, A, dist, str(tune))
        outs[str(tune)] = got
    again = run_gpu(B, A, d, dist, 4, tune={"col_split": 2})
    assert np.array_equal(again, outs[str({"col_split": 2})])


def test_heavy_column_split_auto_and_single_column(B, oracle_lib):
    # n >= 512 turns splitting on by itself; one column holding every row
    m, n, d = 40_000, 600, 140
    rng = np.random.default_rng(9)
    er, ec = rng.integers(0, m, 5000), rng.integers(0, n, 5000)
    key = np.unique(ec[ec != 17] * m + er[ec != 17])
    rows = np.concatenate([np.arange(m), key % m])
    cols = np.concatenate([np.full(m, 17), key // m])
    A = inputs.from_coo(m, n, rows, cols, rng.standard_normal(rows.size).astype(np.float32))
    for dist in DISTS:
        print(f"single heavy column {dist}", flush=True)
        ref = run_oracle(oracle_lib, A, d, dist, 2)
        for tune in [None, {"col_split": 1}]:
            assert_parity(run_gpu(B, A, d, dist, 2, tune=tune), ref, A, dist, str(tune))


@pytest.mark.parametrize("dist", DISTS)
def test_row_weight_mix(B, oracle_lib, dist):
    # a few full rows among light ones: blocks are cut by entry count, a row
    # heavier than the staging capacity forms a block of its own (several
    # staging passes), and the dense path takes the full rows
    m, n, d = 20_000, 1500, 96
    rng = np.random.default_rng(12)
    heavy = rng.choice(m, size=30, replace=False)
    light = np.setdiff1d(np.arange(m), heavy)
    lr = np.repeat(light, 2)
    lc = rng.integers(0, n, lr.size)
    key = np.unique(lc * m + lr)
    rows = np.concatenate([key % m, np.repeat(heavy, n)])
    cols = np.concatenate([key // m, np.tile(np.arange(n), heavy.size)])
    A = inputs.from_coo(m, n, rows, cols, rng.uniform(-1, 1, rows.size).astype(np.float32))
    ref = run_oracle(oracle_lib, A, d, dist, 17)
    for tune in [None, {"dense_min_pct": 101}, {"rows_per_block": 1900, "dense_min_pct": 101},
                 {"rows_per_block": 1900, "dense_min_pct": 30}, {"col_split": 1, "splits": 5}]:
        print(f"row mix {dist} {tune}", flush=True)
        got = run_gpu(B, A, d, dist, 17, tune=tune)
        assert_parity(got, ref, A, dist, str(tune))


# --------------------------------------------------------- precision path
@pytest.mark.parametrize("prec", [1, 2])  # BF16, FP8
@pytest.mark.parametrize("m,n,d,row0", [(20_000, 300, 700, 0), (9_001, 77, 203, 45),
                                        (4_000, 129, 64, 128)])
def test_precision_path_against_oracle(B, oracle_lib, prec, m, n, d, row0):
    # +-1 S is exact in BF16 and FP8: on the matrix cores only A's values round;
    # within 1e-2 of the FP64 oracle on U(-1,1) values
    A = inputs.uniform_positions(m, n, int(0.03 * m * n), m + n + prec, "uniform", np.float32)
    ref = run_oracle(oracle_lib, A, d, "rademacher", 31, row0=row0)
    print(f"precision {prec} m={m} n={n} d={d} row0={row0}", flush=True)
    dA = B.DeviceCsc.from_host(A)
    got = B.sketch(dA, d, "rademacher", 31, row0=row0, prec=prec,
                   tune={"dense_min_pct": 1}).cpu().numpy().astype(np.float64)
    norm, _ = rel_errors(got, ref)
    assert norm <= 1e-2, norm
    # values exact in the operand format: the error is that of FP32 sums
    vals = np.where(A.vals >= 0, 1.0, -1.0) * np.where(np.abs(A.vals) > 0.5, 0.5, 0.25)
    Ae = inputs.Csc(A.m, A.n, A.colptr, A.rowidx, vals.astype(np.float32))
    got = B.sketch(B.DeviceCsc.from_host(Ae), d, "rademacher", 31, row0=row0, prec=prec,
                   tune={"dense_min_pct": 1}).cpu().numpy().astype(np.float64)
    assert_parity(got, run_oracle(oracle_lib, Ae, d, "rademacher", 31, row0=row0), Ae,
                  "rademacher", "exact operands")


def test_precision_path_rules(B):
    m, n = 5000, 40
    A = inputs.uniform_positions(m, n, 2000, 4, "uniform", np.float32)
    dA = B.DeviceCsc.from_host(A)
    with pytest.raises(B.SketchError):  # only +-1 S is exact in the narrow formats
        B.sketch(dA, 80, "uniform", 1, prec=1)
    # below the density threshold the FP32 sparse kernel runs (same result as
    # prec 0 with the same tuning; with no tuning this tiny shape would take
    # the Algorithm 3 kernel, another summation order)
    a = B.sketch(dA, 80, "rademacher", 1, prec=1, tune={"dense_min_pct": 50}).cpu().numpy()
    b = B.sketch(dA, 80, "rademacher", 1, prec=0, tune={"dense_min_pct": 50}).cpu().numpy()
    assert np.array_equal(a, b)


def test_unaligned_row_indices(B, oracle_lib):
    # row indices and values that start 4 bytes past a 16-byte boundary (a
    # view into a larger tensor): the block-position search then reads its
    # windows one entry at a time; the result must not depend on it
    import torch
    A = inputs.uniform_positions(30_000, 60, 60_000, 3, "uniform", np.float32)
    aligned = B.DeviceCsc.from_host(A)
    big_r = torch.zeros(A.nnz + 1, dtype=torch.int32, device="cuda")
    big_v = torch.zeros(A.nnz + 1, dtype=torch.float32, device="cuda")
    big_r[1:] = aligned.rowidx
    big_v[1:] = aligned.vals
    shifted = B.DeviceCsc(A.m, A.n, aligned.colptr, big_r[1:], big_v[1:])
    assert shifted.rowidx.data_ptr() % 16 == 4
    for dist in DISTS:
        a = B.sketch(aligned, 150, dist, 9).cpu().numpy()
        s = B.sketch(shifted, 150, dist, 9).cpu().numpy()
        assert np.array_equal(a, s), dist
        assert_parity(s.astype(np.float64), run_oracle(oracle_lib, A, 150, dist, 9), A, dist,
                      "unaligned")


# ------------------------------------------------- generator call count
def expected_calls(R, row0, d, d_b, e):
    """Generator calls of a sketch whose every row block regenerates its S
    tiles once: each nonempty row of A is generated once per S-row tile, one
    call per group of e S rows (e = 128 for +-1, 4 otherwise) that the tile's
    rows [row0 + t d_b, row0 + (t + 1) d_b) touch."""
    total = 0
    for t in range(-(-d // d_b)):
        g0 = row0 + t * d_b
        total += (g0 + d_b - 1) // e - g0 // e + 1
    return R * total


@pytest.mark.parametrize("dist", DISTS)
@pytest.mark.parametrize("variant,tile_rows", [(3, 32), (5, 64), (5, 128), (2, 16), (6, 64)])
@pytest.mark.parametrize("row0", [0, 100, 3])
def test_generator_call_count(B, oracle_lib, dist, variant, tile_rows, row0):
    # the S tile of a row block is generated once and reused by every column:
    # the call count is exactly R x (generator groups per tile), summed over
    # the tiles (no dense blocks here)
    import torch
    m, n, d = 7001, 77, 203
    A = inputs.uniform_positions(m, n, 9000, 5, "normal", np.float64)
    R = int(np.unique(A.rowidx).size)
    tune = {"variant": variant, "tile_rows": tile_rows, "rows_per_block": 97,
            "dense_min_pct": 101, "count_rng": 1}
    print(f"call count {dist} variant={variant} d_b={tile_rows} row0={row0}", flush=True)
    dA = B.DeviceCsc.from_host(A)
    ws = B.alloc_workspace(B.workspace_bytes(dA, d, dist, tune=tune))
    out = torch.empty((n, d), dtype=torch.float32, device="cuda")
    B.sketch_into(dA, d, dist, 42, out, ws, row0=row0, tune=tune)
    calls = B.sketch_rng_calls(ws)
    e = 128 if dist == "rademacher" else 4
    assert calls == expected_calls(R, row0, d, tile_rows, e), (calls, R)
    got = out.t().cpu().numpy().astype(np.float64)
    assert_parity(got, run_oracle(oracle_lib, A, d, dist, 42, row0=row0), A, dist, "counted")
    # the product instantiation gives the same A_hat bit for bit
    plain = dict(tune, count_rng=0)
    out2 = torch.empty_like(out)
    B.sketch_into(dA, d, dist, 42, out2, ws, row0=row0, tune=plain)
    assert torch.equal(out, out2)
    assert B.sketch_rng_calls(ws) == 0
