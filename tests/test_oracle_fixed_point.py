"""Pins for the oracle's ILU(0) by synchronous fixed-point sweeps (Section 7:
the fixed-point ILU named for computing the factorization on the GPU).  CPU
only."""
import numpy as np
import pytest

from paper_2111_09512_amd import workloads as W

MATS = {
    "poisson6": lambda: W.poisson7(6),
    "vardens6": lambda: W.vardens7(6, seed_rho=4),
    "aniso5": lambda: W.aniso27(5),
    "mmatrix200": lambda: W.random_mmatrix(200, 0.03, seed=5),
    "perm5": lambda: W.permuted_longrange7(5, seed=1),
}


@pytest.mark.parametrize("name", list(MATS))
def test_fixed_point_is_ilu0_bitwise(orc, name):
    """Swept to a standstill, the fixed point is the row-wise ILU(0), bit for
    bit (same products, subtracted in the same ascending order)."""
    A = MATS[name]()
    Ls, U, k = orc.ilu0_fixed_point(A, 2000)
    assert k <= 2000
    Ls0, U0 = orc.ilu0(A)
    for got, ref in ((Ls, Ls0), (U, U0)):
        np.testing.assert_array_equal(got.row_ptr, ref.row_ptr)
        np.testing.assert_array_equal(got.col, ref.col)
        np.testing.assert_array_equal(got.val, ref.val)


@pytest.mark.parametrize("name", ["poisson6", "mmatrix200"])
def test_fixed_point_satisfies_its_equations(orc, name):
    """Independent of the row-wise code: (L U)_ij = a_ij on the pattern of A,
    checked densely."""
    A = MATS[name]()
    Ls, U, k = orc.ilu0_fixed_point(A, 2000)
    LU = (np.eye(A.n) + Ls.to_dense()) @ U.to_dense()
    Ad = A.to_dense()
    mask = Ad != 0
    np.testing.assert_allclose(LU[mask], Ad[mask], rtol=1e-12, atol=1e-12)


def test_initial_guess_and_one_sweep_by_hand(orc):
    """A = [[4, 1, 0], [2, 5, 1], [0, 3, 6]]: the guess is u = a, l_ij = a_ij / a_jj;
    one sweep gives u_11 = 5 - (2/4)*1 = 4.5, l_21 = 3/5 (guess u_11 = 5),
    u_22 = 6 - (3/5)*1 = 5.4; l_10 = 2/4 and the first row are already exact."""
    A = W.CSR.from_dense(np.array([[4.0, 1.0, 0.0], [2.0, 5.0, 1.0], [0.0, 3.0, 6.0]]))
    Ls, U, _ = orc.ilu0_fixed_point(A, 0)
    np.testing.assert_array_equal(Ls.val, [2.0 / 4.0, 3.0 / 5.0])
    np.testing.assert_array_equal(U.val, [4.0, 1.0, 5.0, 1.0, 6.0])
    Ls, U, _ = orc.ilu0_fixed_point(A, 1)
    np.testing.assert_allclose(Ls.val, [0.5, 0.6], rtol=1e-15)
    np.testing.assert_allclose(U.val, [4.0, 1.0, 4.5, 1.0, 5.4], rtol=1e-15)
    Ls, U, k = orc.ilu0_fixed_point(A, 10)  # second sweep fixes l_21 = 3 / 4.5
    np.testing.assert_allclose(Ls.val, [0.5, 3.0 / 4.5], rtol=1e-15)
    np.testing.assert_allclose(U.val[-1], 6.0 - (3.0 / 4.5) * 1.0, rtol=1e-15)
    assert k == 3


def test_residual_shrinks_with_sweeps(orc):
    """The fixed-point residual on the pattern, ||(A - L U)_S||_F, falls as the
    sweeps proceed and is ~0 at the standstill."""
    A = MATS["vardens6"]()
    Ad = A.to_dense()
    mask = Ad != 0
    res = []
    for s in (0, 2, 4, 8, 16):
        Ls, U, _ = orc.ilu0_fixed_point(A, s)
        LU = (np.eye(A.n) + Ls.to_dense()) @ U.to_dense()
        res.append(np.linalg.norm((LU - Ad)[mask]) / np.linalg.norm(Ad[mask]))
    assert res[-1] < 1e-3 * res[0]
    assert res[1] < res[0]


def test_missing_diagonal(orc):
    A = W.CSR.from_dense(np.array([[2.0, 0.0], [1.0, 0.0]]))
    A.val[:] = [2.0, 1.0]
    with pytest.raises(orc.OracleError):
        orc.ilu0_fixed_point(A, 3)
