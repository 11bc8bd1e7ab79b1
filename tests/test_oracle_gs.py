"""Pins for the oracle's polynomial Gauss-Seidel smoother (Section 2: the
polynomial smoother the ILU smoother is compared with): Gauss-Seidel's
(D + L)^{-1} written as (I + D^{-1}L)^{-1} D^{-1}, the inverse replaced by an
m-term Neumann series.  CPU only."""
import numpy as np
import pytest
import scipy.linalg as sla

from paper_2111_09512_amd import workloads as W


def _dense(M):
    return M.to_dense()


def test_split_definition(orc):
    """Gs = D^{-1} L entry by entry (one division), dinv = 1/a_ii, and
    D (I + Gs) reproduces tril(A)."""
    A = W.random_mmatrix(80, 0.1, seed=1)
    Gs, dinv = orc.gs_split(A)
    Ad = _dense(A)
    d = np.diag(Ad)
    np.testing.assert_array_equal(dinv, 1.0 / d)
    G = _dense(Gs)
    assert np.all(np.triu(G) == 0.0)
    rows, cols = np.nonzero(np.tril(Ad, -1))
    np.testing.assert_array_equal(G[rows, cols], Ad[rows, cols] / d[rows])
    assert Gs.nnz == len(rows)
    np.testing.assert_allclose(d[:, None] * (np.eye(A.n) + G), np.tril(Ad), rtol=1e-15, atol=0)


@pytest.mark.parametrize("m", [1, 2, 3, 6])
def test_dense_neumann_formula(orc, m):
    """x1 = x0 + sum_{j<m} (-D^{-1}L)^j D^{-1} (b - A x0), by dense powers."""
    A = W.random_mmatrix(60, 0.12, seed=3)
    Gs, dinv = orc.gs_split(A)
    b, x0 = W.rhs(A.n, 1), W.rhs(A.n, 2)
    Ad = _dense(A)
    D = np.diag(np.diag(Ad))
    Lo = np.tril(Ad, -1)
    Nm = -np.linalg.solve(D, Lo)
    r = np.linalg.solve(D, b - Ad @ x0)
    ref = x0.copy()
    term = r.copy()
    for _ in range(m):
        ref = ref + term
        term = Nm @ term
    got = orc.gs_smooth(A, Gs, dinv, b, x0, 1, m)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13)


def test_many_terms_is_gauss_seidel(orc):
    """With at least depth(L) terms the series is exact: one step is the
    Gauss-Seidel update x + (D + L)^{-1}(b - A x)."""
    A = W.poisson7(5)
    Gs, dinv = orc.gs_split(A)
    depth = orc.levels(Gs, "L")[1]
    b, x0 = W.rhs(A.n, 0), W.rhs(A.n, 4)
    Ad = _dense(A)
    ref = x0 + sla.solve_triangular(np.tril(Ad), b - Ad @ x0, lower=True)
    got = orc.gs_smooth(A, Gs, dinv, b, x0, 1, depth)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13)
    # one term fewer is not exact
    short = orc.gs_smooth(A, Gs, dinv, b, x0, 1, depth - 1)
    assert np.abs(short - ref).max() > 1e-10


def test_one_term_is_jacobi(orc):
    A = W.vardens7(6, seed_rho=2)
    Gs, dinv = orc.gs_split(A)
    b, x0 = W.rhs(A.n, 3), W.rhs(A.n, 5)
    r = orc.residual(A, b, x0)
    np.testing.assert_array_equal(orc.gs_smooth(A, Gs, dinv, b, x0, 1, 1), x0 + dinv * r)


def test_exact_gauss_seidel_converges(orc):
    """Gauss-Seidel converges on a symmetric positive definite matrix:
    repeated exact steps drive the relative residual below 1e-8."""
    A = W.poisson7(6)
    Gs, dinv = orc.gs_split(A)
    depth = orc.levels(Gs, "L")[1]
    b = W.rhs(A.n, 0)
    x = np.zeros(A.n)
    hist = []
    for _ in range(400):
        x = orc.gs_smooth(A, Gs, dinv, b, x, 1, depth)
        hist.append(np.linalg.norm(orc.residual(A, b, x)) / np.linalg.norm(b))
        if hist[-1] < 1e-8:
            break
    assert hist[-1] < 1e-8 and np.all(np.diff(hist) < 0)


def test_mixed_within_fp32(orc):
    A = W.vardens7(8, seed_rho=6)
    Gs, dinv = orc.gs_split(A)
    b = W.rhs(A.n, 4)
    x64 = orc.gs_smooth(A, Gs, dinv, b, np.zeros(A.n), 2, 4)
    x32 = orc.gs_smooth(A, Gs, dinv, b, np.zeros(A.n), 2, 4, mixed=True)
    assert not np.array_equal(x32, x64)
    np.testing.assert_allclose(x32, x64, rtol=0, atol=1e-5 * np.abs(x64).max())


def test_split_errors(orc):
    A = W.CSR.from_dense(np.array([[2.0, 0.0], [1.0, 0.0]]))
    A.val[:] = [2.0, 1.0]  # row 1 stores no diagonal
    with pytest.raises(orc.OracleError):
        orc.gs_split(A)
    B = W.CSR.from_dense(np.array([[2.0, 1.0], [1.0, 3.0]]))
    B.val[3] = 0.0
    with pytest.raises(orc.OracleError):
        orc.gs_split(B)
