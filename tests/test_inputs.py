"""The synthetic stand-ins for the paper's matrices have the stated shapes,
nonzero counts and patterns (host only)."""
import numpy as np
import pytest

from paper_2310_15419_amd import inputs


@pytest.mark.parametrize("name", list(inputs.TABLE1))
def test_table1_standins(name):
    m, n, nnz = inputs.TABLE1[name]
    A, d = inputs.table1_standin(name)
    assert (A.m, A.n, A.nnz, d) == (m, n, nnz, 3 * n)
    per_row = np.bincount(A.rowidx, minlength=m)
    assert per_row.min() == nnz // m and per_row.max() <= nnz // m + 1
    for k in range(0, n, max(1, n // 50)):  # sorted, distinct rows within columns
        r = A.rowidx[A.colptr[k]:A.colptr[k + 1]]
        assert np.all(np.diff(r) > 0)


def test_abnormal_patterns():
    m, n = 20_000, 3_000
    a = inputs.abnormal("A", m, n)
    rows = np.unique(a.rowidx)
    assert np.array_equal(rows, np.arange(0, m, 1000)) and a.nnz == rows.size * n
    c = inputs.abnormal("C", m, n)
    cols = np.flatnonzero(np.diff(c.colptr))
    assert np.array_equal(cols, np.arange(0, n, 1000)) and c.nnz == cols.size * m
    b = inputs.abnormal("B", m, n)
    assert b.nnz == round(1e-3 * m * n)
    owner = np.repeat(np.arange(n), np.diff(b.colptr))
    mid = (owner >= n // 3) & (owner < 2 * n // 3)
    assert abs(mid.mean() - 2998 / 3000) < 1e-3
