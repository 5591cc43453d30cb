"""Pins for the oracle's A_hat = S A (CPU only).

Brute force (numpy matmul of the explicit S with the dense A), identity blocks
(A_hat columns equal scaled S columns exactly), panel-width independence,
linearity / column concatenation / row stacking through row0, the second
moment E[A_hat^T A_hat] = d sigma^2 A^T A, and the subspace-embedding bound
cond <= (sqrt(g)+1)/(sqrt(g)-1) for d = g n (experiments section, gamma = 2).
"""
import numpy as np
import pytest

from paper_2310_15419_amd import inputs

DISTS = ["rademacher", "uniform", "gaussian"]


def _rand_csc(m, n, nnz, seed, dist="normal"):
    return inputs.uniform_positions(m, n, nnz, seed, dist, np.float64)


@pytest.mark.parametrize("dist", DISTS)
@pytest.mark.parametrize("row0", [0, 77, 130])
def test_brute_force(oracle_lib, dist, row0):
    m, n, d = 1500, 40, 200
    A = _rand_csc(m, n, 3000, 1 + row0)
    Ah = oracle_lib.sketch(m, n, A.colptr, A.rowidx, A.vals, d, dist, 9, row0=row0)
    S = oracle_lib.materialize_s(dist, 9, row0, d, 0, m)
    ref = S @ A.to_dense()
    assert np.max(np.abs(Ah - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("dist", DISTS)
def test_identity_blocks_exact(oracle_lib, dist):
    # one entry 2^e per column at distinct rows p_k: A_hat[:, k] = 2^e S[:, p_k] exactly
    m, n, d = 5000, 60, 150
    rng = np.random.default_rng(2)
    p = rng.choice(m, size=n, replace=False)
    e = rng.integers(-3, 4, size=n)
    A = inputs.from_coo(m, n, p, np.arange(n), 2.0 ** e)
    Ah = oracle_lib.sketch(m, n, A.colptr, A.rowidx, A.vals, d, dist, 4)
    for k in range(n):
        col = oracle_lib.materialize_s(dist, 4, 0, d, int(p[k]), 1)[:, 0]
        assert np.array_equal(Ah[:, k], (2.0 ** e[k]) * col)


@pytest.mark.parametrize("dist", DISTS)
def test_panel_width_is_bitwise_irrelevant(oracle_lib, dist):
    m, n, d = 3000, 30, 64
    A = _rand_csc(m, n, 4000, 3)
    whole = oracle_lib.sketch(m, n, A.colptr, A.rowidx, A.vals, d, dist, 8, panel=m)
    for pw in (1, 7, 256, 2999):
        part = oracle_lib.sketch(m, n, A.colptr, A.rowidx, A.vals, d, dist, 8, panel=pw)
        assert np.array_equal(whole, part)


def test_concatenation_and_row_stacking(oracle_lib):
    m, d = 2000, 96
    A1 = _rand_csc(m, 17, 900, 5)
    A2 = _rand_csc(m, 11, 700, 6)
    cat = inputs.from_coo(m, 28,
                          np.concatenate([_rows(A1), _rows(A2)]),
                          np.concatenate([_cols(A1), _cols(A2) + 17]),
                          np.concatenate([A1.vals, A2.vals]))
    for dist in DISTS:
        s1 = oracle_lib.sketch(m, 17, A1.colptr, A1.rowidx, A1.vals, d, dist, 12)
        s2 = oracle_lib.sketch(m, 11, A2.colptr, A2.rowidx, A2.vals, d, dist, 12)
        sc = oracle_lib.sketch(m, 28, cat.colptr, cat.rowidx, cat.vals, d, dist, 12)
        assert np.array_equal(sc, np.concatenate([s1, s2], axis=1))
        # rows [0, d) == rows [0, 40) stacked on rows [40, d) via row0
        top = oracle_lib.sketch(m, 17, A1.colptr, A1.rowidx, A1.vals, 40, dist, 12)
        bot = oracle_lib.sketch(m, 17, A1.colptr, A1.rowidx, A1.vals, d - 40, dist, 12, row0=40)
        assert np.array_equal(s1, np.concatenate([top, bot], axis=0))


def test_linearity(oracle_lib):
    m, n, d = 2500, 20, 80
    A = _rand_csc(m, n, 2000, 21)
    B = inputs.from_coo(m, n, _rows(A), _cols(A), np.random.default_rng(0).standard_normal(A.nnz))
    C = inputs.from_coo(m, n, _rows(A), _cols(A), 2.5 * A.vals - B.vals)
    for dist in DISTS:
        sa = oracle_lib.sketch(m, n, A.colptr, A.rowidx, A.vals, d, dist, 3)
        sb = oracle_lib.sketch(m, n, B.colptr, B.rowidx, B.vals, d, dist, 3)
        sc = oracle_lib.sketch(m, n, C.colptr, C.rowidx, C.vals, d, dist, 3)
        assert np.allclose(sc, 2.5 * sa - sb, rtol=0, atol=1e-12 * np.abs(sa).max())


def _rows(A):
    return A.rowidx.astype(np.int64)


def _cols(A):
    return np.repeat(np.arange(A.n), np.diff(A.colptr))


@pytest.mark.parametrize("dist,sigma2", [("rademacher", 1.0), ("uniform", 1 / 3), ("gaussian", 1.0)])
def test_second_moment(oracle_lib, dist, sigma2):
    # E[A_hat^T A_hat] = d sigma^2 A^T A (unscaled sketch)
    m, n, d, K = 40, 4, 8, 4000
    A = _rand_csc(m, n, 60, 99)
    G = A.to_dense().T @ A.to_dense()
    samples = np.empty((K, n, n))
    for s in range(K):
        Ah = oracle_lib.sketch(m, n, A.colptr, A.rowidx, A.vals, d, dist, 1000 + s)
        samples[s] = Ah.T @ Ah
    mean = samples.mean(axis=0)
    se = samples.std(axis=0, ddof=1) / np.sqrt(K)
    assert np.all(np.abs(mean - d * sigma2 * G) <= 5 * se + 1e-9)


@pytest.mark.parametrize("dist", DISTS)
def test_subspace_embedding_condition(oracle_lib, dist):
    # d = 2n: cond(A R^-1) <= (sqrt2+1)/(sqrt2-1) ~ 5.83 asymptotically; allow 7
    m, n, d = 3000, 200, 400
    Q, _ = np.linalg.qr(np.random.default_rng(7).standard_normal((m, n)))
    rows = np.repeat(np.arange(m), n)
    cols = np.tile(np.arange(n), m)
    A = inputs.from_coo(m, n, rows, cols, Q.ravel())
    Ah = oracle_lib.sketch(m, n, A.colptr, A.rowidx, A.vals, d, dist, 17)
    sv = np.linalg.svd(Ah, compute_uv=False)
    assert sv[0] / sv[-1] <= 7.0
    R = np.linalg.qr(Ah, mode="r")
    assert np.linalg.cond(Q @ np.linalg.inv(R)) <= 7.0


def test_rejects_malformed(oracle_lib):
    A = _rand_csc(100, 5, 50, 1)
    bad = A.rowidx.copy()
    lo = A.colptr[2]
    bad[lo], bad[lo + 1] = bad[lo + 1], bad[lo]
    with pytest.raises(ValueError):
        oracle_lib.sketch(100, 5, A.colptr, bad, A.vals, 8, "uniform", 1)
    bad2 = A.rowidx.copy()
    bad2[0] = 100
    with pytest.raises(ValueError):
        oracle_lib.sketch(100, 5, A.colptr, bad2, A.vals, 8, "uniform", 1)


def test_nonempty_rows_expectation():
    # E[#nonempty rows] = m (1 - (1 - rho)^n) for uniform density rho (Sec. III-A)
    m, n, rho = 100_000, 200, 0.01
    counts = [np.unique(inputs.uniform_positions(m, n, int(rho * m * n), s).rowidx).size
              for s in range(5)]
    expect = m * (1 - (1 - rho) ** n)
    # per-sample sd <= sqrt(m p (1-p)), p = 1-(1-rho)^n
    p = 1 - (1 - rho) ** n
    assert abs(np.mean(counts) - expect) < 5 * np.sqrt(m * p * (1 - p) / 5) + 50


def test_parity_measures_by_brute_force(oracle_lib):
    # the error measures on a tiny case, recomputed element by element
    from paper_2310_15419_amd import inputs
    A = inputs.uniform_positions(50, 4, 30, 2, "normal", np.float64)
    rng = np.random.default_rng(0)
    ref = rng.standard_normal((6, 4))
    got = ref + 1e-3 * rng.standard_normal((6, 4))
    p = oracle_lib.parity(got, ref, A.colptr, A.vals, "gaussian")
    smax = np.sqrt(-2.0 * np.log(2.0**-24))
    worst = 0.0
    for k in range(4):
        s = sum(abs(A.vals[e]) for e in range(A.colptr[k], A.colptr[k + 1])) * smax
        for i in range(6):
            e = abs(got[i, k] - ref[i, k])
            worst = max(worst, e / s if s > 0 else e)
    assert np.isclose(p["max_elem_scaled"], worst, rtol=1e-12)
    assert np.isclose(p["normwise"], np.sqrt(((got - ref) ** 2).sum() / (ref ** 2).sum()))
    cols = [np.sqrt(((got[:, k] - ref[:, k]) ** 2).sum() / (ref[:, k] ** 2).sum())
            for k in range(4)]
    assert np.isclose(p["max_col"], max(cols))
    assert p["nonfinite"] == 0
