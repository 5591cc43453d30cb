"""The Algorithm 3 (kji) loop-order kernel against the oracle, and both
kernels on stand-ins for the paper's SpMM workloads (Table I shapes at full
size; the Table VI patterns at a tenth of their size)."""
import numpy as np
import pytest

from paper_2310_15419_amd import inputs

pytestmark = pytest.mark.gpu

DISTS = ["rademacher", "uniform", "gaussian"]


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    from paper_2310_15419_amd import binding
    binding.lib()
    return binding


def check(oracle_lib, got, A, d, dist, seed, row0=0, what=""):
    ref = oracle_lib.sketch(A.m, A.n, A.colptr, A.rowidx, A.vals.astype(np.float64), d, dist,
                            seed, row0=row0)
    p = oracle_lib.parity(np.asarray(got, dtype=np.float64), ref, A.colptr, A.vals, dist)
    print(f"{what}: {p}", flush=True)
    assert p["nonfinite"] == 0 and p["normwise"] <= 1e-5 and p["max_col"] <= 1e-4, p
    assert p["max_elem_scaled"] <= oracle_lib.ELEM_TOL, p


@pytest.mark.parametrize("dist", DISTS)
@pytest.mark.parametrize("row0,d", [(0, 203), (3, 300), (100, 2100), (64, 5000)])
def test_colwise_against_oracle(B, oracle_lib, dist, row0, d):
    # tiles of 256 (2048 for +-1) rows with ragged tails; row offsets that
    # split a generator group or a 32-row word
    A = inputs.uniform_positions(9001, 57, 12_000, 4, "normal", np.float64)
    got = B.sketch_colwise(B.DeviceCsc.from_host(A), d, dist, 42, row0=row0).cpu().numpy()
    check(oracle_lib, got, A, d, dist, 42, row0, f"colwise {dist} row0={row0} d={d}")


def test_colwise_edges_and_validation(B, oracle_lib):
    import torch
    # empty columns, one entry, a single dense column
    m, n = 3000, 6
    rows = np.concatenate([np.arange(m), [5]])
    cols = np.concatenate([np.full(m, 2), [4]])
    A = inputs.from_coo(m, n, rows, cols, np.linspace(-1, 1, rows.size).astype(np.float32))
    for dist in DISTS:
        got = B.sketch_colwise(B.DeviceCsc.from_host(A), 130, dist, 7).cpu().numpy()
        check(oracle_lib, got, A, 130, dist, 7, 0, f"edges {dist}")
    # unsorted rows in a column: status and NaN
    r = A.rowidx.copy()
    r[10], r[11] = r[11], r[10]
    bad = B.DeviceCsc(m, n, torch.from_numpy(A.colptr).cuda(), torch.from_numpy(r).cuda(),
                      torch.from_numpy(A.vals).cuda())
    with pytest.raises(B.SketchError) as e:
        B.sketch_colwise(bad, 64, "uniform", 1)
    assert e.value.code == -2
    out = B.sketch_colwise(bad, 64, "uniform", 1, check=False)
    assert torch.isnan(out).all()


@pytest.mark.parametrize("name", ["mk-12", "cis-n4c6-b4"])
def test_table1_standins_both_kernels(B, oracle_lib, name):
    # the Table I shapes at full size, d = 3n, (-1,1) S as in the paper's tables
    A, d = inputs.table1_standin(name)
    dA = B.DeviceCsc.from_host(A)
    print(f"{name}: m={A.m} n={A.n} nnz={A.nnz} d={d}", flush=True)
    tile = B.sketch(dA, d, "uniform", 5).cpu().numpy()
    check(oracle_lib, tile, A, d, "uniform", 5, 0, f"{name} S-tile kernel")
    col = B.sketch_colwise(dA, d, "uniform", 5).cpu().numpy()
    check(oracle_lib, col, A, d, "uniform", 5, 0, f"{name} kji kernel")


@pytest.mark.parametrize("kind", ["A", "B", "C"])
def test_abnormal_patterns_both_kernels(B, oracle_lib, kind):
    # Table VI's patterns at a tenth of m and n (the same density), d = 3n
    A = inputs.abnormal(kind, m=10_000, n=1_000)
    d = 3 * A.n
    dA = B.DeviceCsc.from_host(A)
    print(f"abnormal {kind}: nnz={A.nnz}", flush=True)
    tile = B.sketch(dA, d, "uniform", 9).cpu().numpy()
    check(oracle_lib, tile, A, d, "uniform", 9, 0, f"abnormal {kind} S-tile kernel")
    col = B.sketch_colwise(dA, d, "uniform", 9).cpu().numpy()
    check(oracle_lib, col, A, d, "uniform", 9, 0, f"abnormal {kind} kji kernel")


@pytest.mark.parametrize("dist", DISTS)
def test_colwise_heavy_columns_in_chunks(B, oracle_lib, dist):
    # columns of 512 (one chunk), 513 (two, the second of one entry), 1024
    # (two full chunks), 5000 (ten) nonzeros, an empty one and a short one;
    # d over several tiles with a ragged tail
    m = 20_000
    rng = np.random.default_rng(17)
    lens = [512, 0, 513, 3, 1024, 5000]
    rows, cols = [], []
    for k, ln in enumerate(lens):
        rows.append(np.sort(rng.choice(m, size=ln, replace=False)))
        cols.append(np.full(ln, k))
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    A = inputs.from_coo(m, len(lens), rows, cols, rng.standard_normal(rows.size))
    dA = B.DeviceCsc.from_host(A)
    for d, row0 in ((700, 0), (2100, 37)):
        print(f"heavy columns {dist} d={d}", flush=True)
        got = B.sketch_colwise(dA, d, dist, 9, row0=row0).cpu().numpy()
        check(oracle_lib, got, A, d, dist, 9, row0, f"heavy {dist} d={d}")
        got64 = B.sketch_colwise_f64(dA, d, dist, 9, row0=row0).cpu().numpy()
        ref = oracle_lib.sketch(A.m, A.n, A.colptr, A.rowidx, A.vals, d, dist, 9, row0=row0)
        col = np.abs(A.to_dense()).sum(axis=0)[None, :]
        smax = oracle_lib.S_MAX[oracle_lib.DIST_NAMES[dist]]
        assert np.all(np.abs(got64 - ref) <= 1e-13 * col * smax)


def test_colwise_longer_chunks_at_large_d(B, oracle_lib):
    # nnz * d large enough that the chunk length doubles (the partials of
    # 512-entry chunks would pass 256 MiB): four columns of 10000 nonzeros,
    # d = 300000; checked on the first and last 3000 rows (the oracle
    # sketches any row range through row0)
    m, n, d = 50_000, 4, 300_000
    rng = np.random.default_rng(23)
    rows = np.concatenate([np.sort(rng.choice(m, size=10_000, replace=False)) for _ in range(n)])
    cols = np.repeat(np.arange(n), 10_000)
    A = inputs.from_coo(m, n, rows, cols, rng.uniform(-1, 1, rows.size))
    got = B.sketch_colwise(B.DeviceCsc.from_host(A), d, "uniform", 4).cpu().numpy()
    for r0 in (0, d - 3000):
        ref = oracle_lib.sketch(A.m, A.n, A.colptr, A.rowidx, A.vals, 3000, "uniform", 4,
                                row0=r0)
        p = oracle_lib.parity(got[r0:r0 + 3000].astype(np.float64), ref, A.colptr, A.vals,
                              "uniform")
        print(f"rows {r0}..: {p}", flush=True)
        assert p["nonfinite"] == 0 and p["max_elem_scaled"] <= oracle_lib.ELEM_TOL, p
