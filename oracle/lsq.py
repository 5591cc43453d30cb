"""Plain numpy/scipy oracle for the sketch-and-precondition least-squares solve
(paper Sec. V-E): QR of the sketch A_hat = S A, then LSQR on A R^{-1}; or, for
problems with singular values near zero, the SVD of the sketch with the
singular values below sigma_max / 1e12 dropped, then LSQR on A V_r S_r^{-1}.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Library routines
(numpy's QR, scipy's LSQR) serve as steps; nothing here is blocked or fused.
"""
from __future__ import annotations

import numpy as np


def ls_error(A, x, b) -> float:
    """Error(x) = ||A^T (A x - b)||_2 / (||A||_F ||A x - b||_2)  (Sec. V-E-2)."""
    r = A @ x - b
    if hasattr(A, "multiply"):
        fro = float(np.sqrt(A.multiply(A).sum()))
    else:
        fro = float(np.linalg.norm(A))
    return float(np.linalg.norm(A.T @ r) / (fro * np.linalg.norm(r)))


def sap_solve_reference(A, b, Ahat, tol: float = 1e-10, maxiter: int = 1000):
    """x = R^{-1} y, y = LSQR(A R^{-1}, b), R from the QR of the sketch.

    Returns (x, iterations, R)."""
    from scipy.sparse.linalg import LinearOperator, lsqr
    from scipy.linalg import solve_triangular

    R = np.linalg.qr(np.asarray(Ahat, dtype=np.float64), mode="r")
    n = R.shape[1]
    m = A.shape[0]

    def mv(v):
        return A @ solve_triangular(R, np.asarray(v).ravel(), lower=False)

    def rmv(u):
        return solve_triangular(R, A.T @ np.asarray(u).ravel(), trans="T", lower=False)

    op = LinearOperator((m, n), matvec=mv, rmatvec=rmv, dtype=np.float64)
    res = lsqr(op, b, atol=tol, btol=tol, iter_lim=maxiter)
    y, itn = res[0], res[2]
    x = solve_triangular(R, y, lower=False)
    return x, itn, R


# Sec. V-E-1: the SVD form drops singular values below sigma_max(S A) / 1e12
SVD_DROP = 1e-12


def sap_svd_reference(A, b, Ahat, tol: float = 1e-10, maxiter: int = 1000,
                      drop: float = SVD_DROP):
    """x = N y, y = LSQR(A N, b), N = V_r diag(1 / sigma_r) from the SVD of the
    sketch A_hat = U diag(sigma) V^T, keeping the r singular values with
    sigma >= drop * sigma_max (Sec. V-E-1).

    Returns (x, iterations, sigma (all, descending), r)."""
    from scipy.sparse.linalg import LinearOperator, lsqr

    _, sig, vt = np.linalg.svd(np.asarray(Ahat, dtype=np.float64), full_matrices=False)
    keep = sig >= drop * sig[0] if sig.size and sig[0] > 0 else np.zeros(sig.size, bool)
    r = int(np.count_nonzero(keep))
    N = vt[keep].T / sig[keep]
    m = A.shape[0]

    def mv(y):
        return A @ (N @ np.asarray(y).ravel())

    def rmv(u):
        return N.T @ (A.T @ np.asarray(u).ravel())

    op = LinearOperator((m, r), matvec=mv, rmatvec=rmv, dtype=np.float64)
    res = lsqr(op, b, atol=tol, btol=tol, iter_lim=maxiter)
    y, itn = res[0], res[2]
    return N @ y, itn, sig, r
