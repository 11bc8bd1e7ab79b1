"""Checks on the seeded input generators (CPU only)."""
import numpy as np
import pytest

from paper_2111_09512_amd import workloads as W


def _sym(A):
    S = A.to_scipy()
    return abs(S - S.T).max() == 0


@pytest.mark.parametrize("N", [3, 5, 8])
def test_poisson7_counts_and_rowsums(N):
    A = W.poisson7(N)
    A.validate()
    assert A.nnz == 7 * N**3 - 6 * N**2  # 223,232 at N = 32
    assert _sym(A)
    d = A.to_dense()
    assert np.all(np.diag(d) == 6.0)
    rs = d.sum(1)
    assert np.all(rs >= 0) and np.any(rs == 0) == (N > 2)
    assert 7 * 32**3 - 6 * 32**2 == 223_232


def test_aniso27_counts_weights():
    N = 6
    A = W.aniso27(N)
    A.validate()
    assert A.nnz == (3 * N - 2) ** 3  # 213,847,192 at N = 200
    assert (3 * 200 - 2) ** 3 == 213_847_192
    assert _sym(A)
    d = A.to_dense()
    i = 1 + N * 1 + N * N * 1  # interior point (1,1,1)
    assert d[i, i + N * N] == -1000.0 and d[i, i + 1] == -1.0
    assert d[i, i + 1 + N] == pytest.approx(-0.5)
    assert d[i].sum() == pytest.approx(0.0, abs=1e-9)


def test_vardens7_is_symmetric_mmatrix():
    A = W.vardens7(6)
    A.validate()
    assert _sym(A)
    d = A.to_dense()
    off = d - np.diag(np.diag(d))
    assert np.all(off <= 0) and np.all(np.diag(d) > 0)
    assert np.all(d.sum(1) >= -1e-9 * np.abs(d).max(1))  # diagonally dominant
    vals = -off[off < 0]
    assert vals.max() / vals.min() > 1e6  # coefficients span many orders of magnitude


def test_permuted_longrange7_structure():
    N = 8
    A = W.permuted_longrange7(N, seed=1)
    A.validate()
    assert _sym(A)
    assert A.nnz == 7 * N**3 - 6 * N**2  # replacement keeps the count
    d = A.to_dense()
    assert np.all(np.diag(d) == 6.0)
    small = (d < 0) & (d > -1e-2)
    assert small.sum() == 2 * int(np.floor(0.1 * 3 * N * N * (N - 1)))
    # deterministic in the seed
    B = W.permuted_longrange7(N, seed=1)
    assert np.array_equal(A.col, B.col) and np.array_equal(A.val, B.val)


def test_rhs_seeded():
    assert np.array_equal(W.rhs(10, 0), W.rhs(10, 0))
    b = W.rhs(1000, 0)
    assert -1 <= b.min() and b.max() <= 1


@pytest.mark.parametrize("N", [4, 7, 11])
def test_permuted_fast_construction_equals_coo(N):
    """The padded-table construction of the permuted operator equals a plain
    COO assembly of the same draws, array for array."""
    A = W.permuted_longrange7(N, seed=1)
    B = W.permuted_longrange7(N, seed=1, coo=True)
    assert np.array_equal(A.row_ptr, B.row_ptr)
    assert np.array_equal(A.col, B.col)
    assert np.array_equal(A.val, B.val)
