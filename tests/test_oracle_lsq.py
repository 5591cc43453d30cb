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
