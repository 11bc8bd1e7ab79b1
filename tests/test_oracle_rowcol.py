"""Pins for the oracle's row/column scaling of U (Section 5.1, eq.
rowcolScale; Table 1's last column, named Ruiz scaling in Table 2) and the smoother built on it (CPU only).

The scaling reading: Ruiz steps in the max norm give D_c; the row factor is
then fixed by the unit diagonal the paper requires, d_r,i = 1/(u_ii d_c,i).
So U^ = D_r U D_c = D_c^{-1} U~ D_c, a diagonal similarity of the row-scaled
factor U~ = D^{-1} U, and the truncated Neumann sums on U^ and on U~ give
the same smoother output in exact arithmetic -- the strongest pin below."""
import numpy as np
import pytest

from paper_2111_09512_amd import workloads as W


def _upper(rows):
    return W.CSR.from_dense(np.array(rows, dtype=np.float64))


def test_hand_2x2_one_step(orc):
    """U = [[4, 9], [0, 1]], one Ruiz step by hand: row maxima 9, 1 give
    r = (1/3, 1); column maxima 4, 9 give c = (1/2, 1/3).  Unit diagonal:
    d_r = (1/(4 * 1/2), 1/(1 * 1/3)) = (1/2, 3); u^_01 = 9 * 1/2 * 1/3 = 3/2."""
    dr, dc, Uh, drr = orc.scale_rowcol(_upper([[4, 9], [0, 1]]), iters=1)
    np.testing.assert_allclose(drr, [1 / 3, 1.0], rtol=1e-15)
    np.testing.assert_allclose(dc, [0.5, 1 / 3], rtol=1e-15)
    np.testing.assert_allclose(dr, [0.5, 3.0], rtol=1e-15)
    assert list(Uh.row_ptr) == [0, 1, 1] and list(Uh.col) == [1]
    assert Uh.val[0] == pytest.approx(1.5, rel=1e-15)


def test_hand_2x2_two_steps(orc):
    """Second step on [[2/3, 1], [0, 1/3]]: row maxima 1, 1/3, column maxima
    2/3, 1, so d_c = (sqrt(3/2)/2, 1/3), the Ruiz row factors (1/3, sqrt 3),
    and u^_01 = 9 d_c1 / (4 d_c0) = sqrt(3/2)."""
    dr, dc, Uh, drr = orc.scale_rowcol(_upper([[4, 9], [0, 1]]), iters=2)
    np.testing.assert_allclose(dc, [np.sqrt(1.5) / 2, 1 / 3], rtol=1e-15)
    np.testing.assert_allclose(drr, [1 / 3, np.sqrt(3.0)], rtol=1e-15)
    np.testing.assert_allclose(dr, [1 / (4 * dc[0]), 3.0], rtol=1e-15)
    assert Uh.val[0] == pytest.approx(np.sqrt(1.5), rel=1e-15)


def test_diagonal_U(orc):
    """A diagonal U scales to the identity: U^ has no off-diagonal entries
    and d_r d_c u = 1, so the U step reduces to z = y / u."""
    u = np.array([2.0, -0.5, 8.0, 3.0])
    dr, dc, Uh, _ = orc.scale_rowcol(_upper(np.diag(u)), iters=3)
    assert Uh.nnz == 0
    np.testing.assert_allclose(dr * dc * u, 1.0, rtol=1e-15)


def _factors(orc, A):
    Ls, U = orc.ilu0(A)
    d, dinv, Us = orc.scale_rows(U)
    return Ls, U, dinv, Us


@pytest.mark.parametrize("iters", [0, 1, 5, 12])
def test_unit_diagonal_and_similarity(orc, iters):
    """On an ILU(0) factor of a non-symmetric operator: (u_ii d_r,i) d_c,i = 1
    to rounding, and U^_s equals D_c^{-1} U~_s D_c entry by entry (U~ from
    the row scaling)."""
    A = W.random_mmatrix(300, 0.03, seed=11)
    Ls, U, dinv, Us = _factors(orc, A)
    dr, dc, Uh, _ = orc.scale_rowcol(U, iters=iters)
    diag = U.val[U.row_ptr[:-1]]
    np.testing.assert_allclose((diag * dr) * dc, 1.0, rtol=4e-16, atol=0)
    assert np.array_equal(Uh.row_ptr, Us.row_ptr) and np.array_equal(Uh.col, Us.col)
    rows = np.repeat(np.arange(U.n), np.diff(Us.row_ptr))
    np.testing.assert_allclose(Uh.val, Us.val * dc[Us.col] / dc[rows], rtol=1e-14)
    if iters == 0:
        np.testing.assert_array_equal(dc, 1.0)
    else:  # a genuine column scaling, not a multiple of the identity
        assert dc.max() > 1.5 * dc.min()


def test_ruiz_equilibrates(orc):
    """Ruiz's max-norm iteration drives every row and column maximum of
    D_r U D_c to 1 (its fixed point); checked on a badly scaled triangle."""
    rng = np.random.default_rng(3)
    n = 60
    T = np.triu(np.where(rng.random((n, n)) < 0.2, rng.uniform(-1, 1, (n, n)), 0.0), 1)
    T += np.diag(rng.uniform(0.5, 2, n))
    T = np.diag(10.0 ** rng.uniform(-4, 4, n)) @ T @ np.diag(10.0 ** rng.uniform(-3, 3, n))
    _, dc, _, drr = orc.scale_rowcol(W.CSR.from_dense(T), iters=40)
    S = np.abs(drr[:, None] * T * dc[None, :])
    np.testing.assert_allclose(S.max(axis=1), 1.0, atol=1e-6)
    np.testing.assert_allclose(S.max(axis=0), 1.0, atol=1e-6)


@pytest.mark.parametrize("mL,mU", [(3, 3), (1, 1), (1, 4), (4, 1), (2, 5)])
def test_smoother_equals_row_scaled_one(orc, mL, mU):
    """Similarity invariance: the row/column-scaled smoother gives the
    row-scaled smoother's x (to rounding) for every sweep count."""
    A = W.vardens7(8, seed_rho=4)
    Ls, U, dinv, Us = _factors(orc, A)
    dr, dc, Uh, _ = orc.scale_rowcol(U, iters=5)
    b, x0 = W.rhs(A.n, 1), W.rhs(A.n, 2)
    ref = orc.smooth(A, Ls, Us, dinv, b, x0, 2, mL, mU)
    got = orc.smooth_rowcol(A, Ls, Uh, dr, dc, b, x0, 2, mL, mU)
    np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())


def test_direct_equals_exact_preconditioner(orc):
    """direct: one step from x = 0 is x = (L U)^{-1} b, whatever the scaling."""
    A = W.random_mmatrix(120, 0.05, seed=2)
    Ls, U, dinv, Us = _factors(orc, A)
    dr, dc, Uh, _ = orc.scale_rowcol(U, iters=4)
    b = W.rhs(A.n, 3)
    got = orc.smooth_rowcol(A, Ls, Uh, dr, dc, b, np.zeros(A.n), 1, 1, 1, direct=True)
    M = (np.eye(A.n) + Ls.to_dense()) @ U.to_dense()
    np.testing.assert_allclose(got, np.linalg.solve(M, b), rtol=1e-10, atol=1e-12)


def test_mixed_within_fp32_of_fp64(orc):
    A = W.vardens7(8, seed_rho=6)
    Ls, U, dinv, Us = _factors(orc, A)
    dr, dc, Uh, _ = orc.scale_rowcol(U, iters=5)
    b = W.rhs(A.n, 4)
    x64 = orc.smooth_rowcol(A, Ls, Uh, dr, dc, b, np.zeros(A.n), 1, 3, 3)
    x32 = orc.smooth_rowcol(A, Ls, Uh, dr, dc, b, np.zeros(A.n), 1, 3, 3, mixed=True)
    assert not np.array_equal(x32, x64)
    np.testing.assert_allclose(x32, x64, rtol=0, atol=1e-5 * np.abs(x64).max())


def test_errors(orc):
    with pytest.raises(orc.OracleError):  # zero pivot
        orc.scale_rowcol(_upper([[1.0, 2.0], [0.0, 0.0]]))
    bad = _upper([[1.0, 2.0], [0.0, 1.0]])
    bad.col[:] = [1, 0, 1]  # row 0 does not start with its diagonal
    with pytest.raises(orc.OracleError):
        orc.scale_rowcol(bad)
