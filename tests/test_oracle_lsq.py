"""Pins of the least-squares oracle (sketch-and-precondition, paper Sec. V-E)
against an independent dense solver and the properties the paper states."""
import numpy as np
import pytest

from paper_2310_15419_amd import inputs


def dense_lstsq(A, b):
    return np.linalg.lstsq(A.to_dense(), b, rcond=None)[0]


@pytest.mark.parametrize("dist", ["rademacher", "gaussian"])
@pytest.mark.parametrize("m,n,dense_rows", [(3000, 40, 100), (8000, 90, 300)])
def test_sap_reference_matches_dense_lstsq(oracle_lib, dist, m, n, dense_rows):
    A, b, _ = inputs.ls_request(5 + n, m, n, dense_rows=dense_rows)
    d = 2 * n
    Ahat = oracle_lib.sketch(A.m, A.n, A.colptr, A.rowidx, A.vals, d, dist, 77)
    x, itn, R = oracle_lib.sap_solve_reference(A.to_scipy(), b, Ahat, tol=1e-10)
    xs = dense_lstsq(A, b)
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
    # the preconditioned operator has condition number near that of a
    # subspace embedding with d = 2n (Sec. IV-B: (sqrt 2 + 1)/(sqrt 2 - 1)),
    # so LSQR converges in well under a hundred iterations
    assert 5 <= itn <= 100, itn
    assert np.allclose(np.abs(np.diag(R)), np.abs(np.diag(np.linalg.qr(Ahat, mode="r"))))


def test_ls_error_metric(oracle_lib):
    A, b, _ = inputs.ls_request(3, 2000, 30, dense_rows=100)
    As = A.to_scipy()
    xs = dense_lstsq(A, b)
    # the exact minimiser satisfies the normal equations to rounding: with a
    # residual ~1e-6 of ||b||, rounding alone gives Error ~ u ||b|| / ||r||
    assert oracle_lib.ls_error(As, xs, b) < 1e-9
    # a perturbed point does not; the metric matches its definition on a dense copy
    xp = xs + 1e-4 * np.random.default_rng(0).standard_normal(xs.size)
    Ad = A.to_dense()
    r = Ad @ xp - b
    direct = np.linalg.norm(Ad.T @ r) / (np.linalg.norm(Ad) * np.linalg.norm(r))
    assert oracle_lib.ls_error(As, xp, b) == pytest.approx(direct, rel=1e-10)
    assert direct > 1e-8


def _null_residuals(x, null):
    """x . z for each known null vector z = e_j - sum c_k e_k of A (the minimum-
    norm solution is orthogonal to the null space), relative to ||x||."""
    out = []
    for j, comb in null:
        v = x[j] - sum(c * x[k] for k, c in comb.items())
        z = np.sqrt(1.0 + sum(c * c for c in comb.values()))  # |e_j - sum c_k e_k|
        out.append(abs(v) / z / np.linalg.norm(x))
    return out


def test_rank_deficient_standin_is_exactly_dependent():
    A, b, null = inputs.ls_request_rank_deficient(3, 4000, 30, 24, dense_rows=100)
    D = A.to_dense()
    for j, comb in null:
        want = sum((c * D[:, k] for k, c in comb.items()), np.zeros(A.m))
        assert np.array_equal(D[:, j], want), j
    assert np.linalg.matrix_rank(D) == 24
    # in FP32 too: the values sit on the grid k/1024 and the sums are exact
    D32 = D.astype(np.float32)
    assert np.array_equal(D32.astype(np.float64), D)


@pytest.mark.parametrize("dist", ["rademacher", "gaussian"])
@pytest.mark.parametrize("m,n,rank", [(4000, 30, 24), (9000, 80, 50)])
def test_sap_svd_gives_minimum_norm_solution(oracle_lib, dist, m, n, rank):
    A, b, null = inputs.ls_request_rank_deficient(n + rank, m, n, rank, dense_rows=150)
    d = 2 * n
    Ahat = oracle_lib.sketch(A.m, A.n, A.colptr, A.rowidx, A.vals, d, dist, 7)
    x, itn, sig, r = oracle_lib.sap_svd_reference(A.to_scipy(), b, Ahat, tol=1e-12)
    # the sketch keeps A's rank (an embedding of range(A)); the null directions
    # give singular values at rounding level, far below the drop threshold
    assert r == rank, (r, sig[rank - 1:rank + 1] / sig[0])
    assert sig[rank] <= 1e-14 * sig[0] and sig[rank - 1] >= 1e-6 * sig[0]
    # x is the minimum-norm least-squares solution: orthogonal to every known
    # null vector of A, equal to numpy's SVD-based minimum-norm lstsq
    assert max(_null_residuals(x, null)) <= 1e-10
    xs = np.linalg.lstsq(A.to_dense(), b, rcond=1e-10)[0]
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
    assert oracle_lib.ls_error(A.to_scipy(), x, b) <= 1e-9
    assert 5 <= itn <= 100, itn


def test_sap_svd_drop_threshold_both_sides(oracle_lib):
    m, n, rank = 6000, 40, 30
    d = 2 * n
    # a singular value ~1e-8 of sigma_max is kept: the solution then uses it.
    # A consistent b (no noise): with a residual, the solution's condition
    # number is kappa^2 ~ 1e16 and any two stable solvers differ by ~1e-5
    A, b, null = inputs.ls_request_rank_deficient(9, m, n, rank, dense_rows=150,
                                                  near=2.0 ** -20, noise=0.0)
    Ahat = oracle_lib.sketch(A.m, A.n, A.colptr, A.rowidx, A.vals, d, "gaussian", 3)
    x, itn, sig, r = oracle_lib.sap_svd_reference(A.to_scipy(), b, Ahat, tol=1e-12)
    assert r == rank + 1 and 1e-12 * sig[0] < sig[rank] < 1e-5 * sig[0]
    # LSQR stops at a backward error ~tol of the preconditioned problem, so x
    # is within about kappa * tol of the exact solution (kappa = sigma_max /
    # sigma_r ~ 1e8 here: ~1e-4), and it fits b far better than the solution
    # without the small direction (forced out with a higher threshold)
    D = A.to_dense()
    kappa = sig[0] / sig[r - 1]
    xs = np.linalg.lstsq(D, b, rcond=1e-13)[0]
    assert np.linalg.norm(x - xs) <= 10 * kappa * 1e-12 * np.linalg.norm(xs)
    assert max(_null_residuals(x, null[1:])) <= 1e-8
    xd, _, _, rd = oracle_lib.sap_svd_reference(A.to_scipy(), b, Ahat, tol=1e-12, drop=1e-7)
    assert rd == rank
    res_kept = np.linalg.norm(D @ x - b)
    assert 10 * res_kept <= np.linalg.norm(D @ xd - b)
    assert np.linalg.norm(xd - x) >= 1e-2 * np.linalg.norm(x)
    # one of ~1e-20 of sigma_max is dropped: rank as without it
    A2, b2, null2 = inputs.ls_request_rank_deficient(9, m, n, rank, dense_rows=150,
                                                     near=2.0 ** -60)
    Ahat2 = oracle_lib.sketch(A2.m, A2.n, A2.colptr, A2.rowidx, A2.vals, d, "gaussian", 3)
    x2, _, sig2, r2 = oracle_lib.sap_svd_reference(A2.to_scipy(), b2, Ahat2, tol=1e-12)
    assert r2 == rank and sig2[rank] < 1e-12 * sig2[0]
    xs2 = np.linalg.lstsq(A2.to_dense(), b2, rcond=1e-12)[0]
    assert np.linalg.norm(x2 - xs2) <= 1e-8 * np.linalg.norm(xs2)


@pytest.mark.parametrize("dist", ["rademacher", "uniform"])
def test_sap_svd_equals_qr_form_on_full_rank(oracle_lib, dist):
    A, b, _ = inputs.ls_request(21, 5000, 50, dense_rows=200)
    Ahat = oracle_lib.sketch(A.m, A.n, A.colptr, A.rowidx, A.vals, 100, dist, 5)
    xq, itq, _ = oracle_lib.sap_solve_reference(A.to_scipy(), b, Ahat, tol=1e-12)
    xv, itv, sig, r = oracle_lib.sap_svd_reference(A.to_scipy(), b, Ahat, tol=1e-12)
    assert r == 50
    assert np.linalg.norm(xv - xq) <= 1e-9 * np.linalg.norm(xq)
    # V diag(1/sigma) and R^{-1} precondition equally well: A R^{-1} and A N
    # differ by an orthogonal factor, so LSQR runs the same iterations
    assert abs(itq - itv) <= 2
