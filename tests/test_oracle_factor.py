"""Pins for the oracle's factorizations and row scaling (CPU only).

Each check compares the oracle with something other than itself: a closed
form, a characterization of the factorization that the paper's definitions fix,
scipy's dense LU, or a dense brute-force computation on tiny inputs.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from paper_2111_09512_amd import workloads as W


def dense(M):
    return M.to_dense()


def unit_lower(Ls):
    return Ls.to_dense() + np.eye(Ls.n)


def col_dominant(n, seed, density=0.5):
    """Random nonsymmetric matrix, strictly diagonally dominant by columns, so
    Gaussian elimination with partial pivoting never swaps rows (P = I)."""
    rng = np.random.default_rng(seed)
    M = np.where(rng.random((n, n)) < density, rng.uniform(-1, 1, (n, n)), 0.0)
    np.fill_diagonal(M, 0.0)
    np.fill_diagonal(M, np.abs(M).sum(0) + 1.0 + rng.random(n))
    return W.CSR.from_dense(M)


# --------------------------------------------------------------------------
# ILU(0)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("sym", [False, True])
def test_ilu0_reproduces_A_on_its_pattern(orc, seed, sym):
    """ILU(0) is characterised by (LU)_ij = a_ij for every (i,j) in pattern(A)
    with L, U confined to that pattern (Section 4.2, 'nofill')."""
    A = W.random_mmatrix(40, 0.15, seed, sym=sym)
    Ls, U = orc.ilu0(A)
    Ad = dense(A)
    P = unit_lower(Ls) @ dense(U)
    mask = Ad != 0
    assert np.max(np.abs(P - Ad)[mask]) <= 1e-13 * np.abs(Ad).max()
    # the factors live on the pattern of A, split at the diagonal
    Lpat = np.zeros_like(mask)
    Upat = np.zeros_like(mask)
    rows = np.repeat(np.arange(Ls.n), np.diff(Ls.row_ptr))
    Lpat[rows, Ls.col] = True
    rows = np.repeat(np.arange(U.n), np.diff(U.row_ptr))
    Upat[rows, U.col] = True
    assert np.array_equal(Lpat, np.tril(mask, -1))
    assert np.array_equal(Upat, np.triu(mask))


def test_ilu0_tridiagonal_closed_form(orc):
    """Tridiagonal (-1, 2, -1): ILU(0) is the exact LU (no fill) with
    u_ii = (i+1)/i and l_{i+1,i} = -i/(i+1) (1-based)."""
    n = 60
    A = W.tridiag(n)
    Ls, U = orc.ilu0(A)
    i = np.arange(1, n + 1, dtype=np.float64)
    d, dinv, Us = orc.scale_rows(U)
    np.testing.assert_allclose(d, (i + 1) / i, rtol=1e-14)
    np.testing.assert_allclose(Ls.val, -i[:-1] / (i[:-1] + 1), rtol=1e-14)
    np.testing.assert_allclose(unit_lower(Ls) @ dense(U), dense(A), atol=1e-14)


# --------------------------------------------------------------------------
# ILU(k)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1])
def test_iluk_full_fill_is_exact_lu(orc, seed):
    """ILU(k) with k >= n-1 keeps every fill entry: it is Gaussian elimination
    without pivoting, equal to scipy's LU when partial pivoting does not swap."""
    A = col_dominant(30, seed, density=0.2)
    P, Lref, Uref = sla.lu(dense(A))
    assert np.array_equal(P, np.eye(A.n))
    Ls, U = orc.iluk(A, A.n)
    np.testing.assert_allclose(unit_lower(Ls), Lref, atol=1e-13)
    np.testing.assert_allclose(dense(U), Uref, atol=1e-13 * np.abs(Uref).max())


@pytest.mark.parametrize("N", [4, 5, 7])
def test_iluk1_pattern_on_7pt_grid(orc, N):
    """ILU(1) of the 7-point grid: eliminating with the three lower neighbours
    creates exactly the level-1 fill offsets (x+1,y-1,z), (x+1,y,z-1),
    (x,y+1,z-1) in L (mirrored in U).  Closed-form count
    3N^2(N-1) + 3N(N-1)^2 per strict factor (12,435,840 at N = 128)."""
    A = W.vardens7(N)
    Ls, U = orc.iluk(A, 1)
    n = N**3
    expect = set()
    for i in range(n):
        x, y, z = i % N, (i // N) % N, i // (N * N)
        for dx, dy, dz in [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (1, -1, 0), (1, 0, -1), (0, 1, -1)]:
            if 0 <= x + dx < N and 0 <= y + dy < N and 0 <= z + dz < N:
                expect.add((i, i + dx + N * dy + N * N * dz))
    rows = np.repeat(np.arange(n), np.diff(Ls.row_ptr))
    got = set(zip(rows.tolist(), Ls.col.tolist()))
    assert got == expect
    assert Ls.nnz == 3 * N * N * (N - 1) + 3 * N * (N - 1) ** 2
    assert U.nnz - n == Ls.nnz
    assert 3 * 128 * 128 * 127 + 3 * 128 * 127**2 == 12_435_840


@pytest.mark.parametrize("k", [1, 2])
def test_iluk_reproduces_A_on_level_pattern(orc, k):
    """On its level-k pattern, ILU(k) satisfies (LU)_ij = a_ij (a_ij = 0 at
    fill positions), the defining property of an incomplete factorization
    restricted to a fixed pattern (Section 3.1: numeric phase on the symbolic
    pattern)."""
    A = W.random_mmatrix(50, 0.06, 7)
    Ls, U = orc.iluk(A, k)
    P = unit_lower(Ls) @ dense(U)
    pat = (dense(Ls) != 0) | (dense(U) != 0)
    # structural zeros of the factors cannot be seen through to_dense; rebuild the pattern
    for M in (Ls, U):
        rows = np.repeat(np.arange(M.n), np.diff(M.row_ptr))
        pat[rows, M.col] = True
    Ad = dense(A)
    assert np.max(np.abs(P - Ad)[pat]) <= 1e-13 * np.abs(Ad).max()
    Ls0, _ = orc.iluk(A, 0)
    assert Ls.nnz > Ls0.nnz  # fill appeared


def test_iluk_symmetric_gives_transposed_scaled_factor(orc):
    """For symmetric A, ILU(k) on a symmetric pattern gives U~ = D^{-1}U = L^T,
    which is why Table 1's dep(D^{-1}U) column equals its dep(L) column."""
    for A in (W.poisson7(5), W.vardens7(5)):
        for k in (0, 1):
            Ls, U = orc.iluk(A, k)
            d, dinv, Us = orc.scale_rows(U)
            np.testing.assert_allclose(dense(Us), dense(Ls).T, rtol=1e-12, atol=1e-15)
            assert orc.dep_triangular(Us) == pytest.approx(orc.dep_triangular(Ls), rel=1e-12)


# --------------------------------------------------------------------------
# ILUT(tau, p)
# --------------------------------------------------------------------------

def test_ilut_tau0_full_fill_is_exact_lu(orc):
    A = col_dominant(25, 3, density=0.25)
    P, Lref, Uref = sla.lu(dense(A))
    assert np.array_equal(P, np.eye(A.n))
    Ls, U = orc.ilut(A, 0.0, A.n)
    np.testing.assert_allclose(unit_lower(Ls), Lref, atol=1e-13)
    np.testing.assert_allclose(dense(U), Uref, atol=1e-13 * np.abs(Uref).max())


def test_ilut_huge_tau_keeps_only_the_diagonal(orc):
    A = W.random_mmatrix(30, 0.2, 4)
    Ls, U = orc.ilut(A, 1e30, 10)
    assert Ls.nnz == 0
    assert U.nnz == A.n
    np.testing.assert_array_equal(dense(U), np.diag(np.diag(dense(A))))


def _row_tau(A, tau):
    Ad = dense(A)
    return tau * np.sqrt((Ad**2).sum(1))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ilut_characterization_without_count_limit(orc, seed):
    """With p >= n the threshold rule alone decides, and the result is
    characterised entry by entry (magnitudes in A's units):
      kept (i,j), j >= i:  (LU)_ij = a_ij and |u_ij| >= tau_i (j > i);
      kept (i,j), j < i:   (LU)_ij = a_ij and |l_ij u_jj| >= tau_i;
      every other (i,j):   |(A - LU)_ij| < tau_i (the dropped remainder)."""
    A = W.random_mmatrix(40, 0.15, 10 + seed)
    tau = 0.05
    Ls, U = orc.ilut(A, tau, A.n)
    Ad = dense(A)
    Ld, Ud = unit_lower(Ls), dense(U)
    R = Ad - Ld @ Ud
    ti = _row_tau(A, tau)
    keptL = np.zeros_like(Ad, dtype=bool)
    keptU = np.zeros_like(Ad, dtype=bool)
    for M, kept in ((Ls, keptL), (U, keptU)):
        rows = np.repeat(np.arange(M.n), np.diff(M.row_ptr))
        kept[rows, M.col] = True
    kept = keptL | keptU
    scale = np.abs(Ad).max()
    assert np.max(np.abs(R[kept])) <= 1e-13 * scale
    off = ~kept
    assert np.all(np.abs(R[off]) < (ti[:, None] * np.ones_like(Ad))[off] * (1 + 1e-12))
    # magnitudes of kept entries pass the threshold
    iu, ju = np.nonzero(keptU & ~np.eye(A.n, dtype=bool))
    assert np.all(np.abs(Ud[iu, ju]) >= ti[iu])
    il, jl = np.nonzero(keptL)
    assert np.all(np.abs(Ld[il, jl] * np.diag(Ud)[jl]) >= ti[il] * (1 - 1e-12))
    assert Ls.nnz > 0 and np.count_nonzero(np.tril(Ad, -1)) > 0


def _dense_ilut(Ad, tau, p):
    """Brute force on tiny inputs: ILUT on dense rows, same reading as the oracle."""
    n = Ad.shape[0]
    L = np.eye(n)
    U = np.zeros((n, n))
    Upresent = np.zeros((n, n), dtype=bool)
    for i in range(n):
        w = Ad[i].copy()
        present = Ad[i] != 0
        present[i] = True
        tau_i = tau * np.sqrt(np.sum(Ad[i][present] ** 2))
        pre = np.zeros(n)
        dropped = np.zeros(n, dtype=bool)
        for k in range(i):
            if not present[k]:
                continue
            v = w[k]
            if abs(v) < tau_i:
                w[k] = 0.0
                dropped[k] = True
                continue
            w[k] = v / U[k, k]
            pre[k] = v
            for j in range(k + 1, n):
                if Upresent[k, j] and j != k:
                    if not present[j]:
                        present[j] = True
                        w[j] = 0.0
                    w[j] -= w[k] * U[k, j]
        lc = [k for k in range(i) if present[k] and not dropped[k]]
        lc = sorted(lc, key=lambda k: (-abs(pre[k]), k))[:p]
        for k in lc:
            L[i, k] = w[k]
        uc = [j for j in range(i + 1, n) if present[j] and abs(w[j]) >= tau_i]
        uc = sorted(uc, key=lambda j: (-abs(w[j]), j))[:p]
        U[i, i] = w[i]
        Upresent[i, i] = True
        for j in uc:
            U[i, j] = w[j]
            Upresent[i, j] = True
    return L, U


@pytest.mark.parametrize("seed,tau,p", [(0, 0.02, 3), (1, 0.01, 2), (2, 0.0, 4), (3, 0.05, 1)])
def test_ilut_matches_dense_bruteforce(orc, seed, tau, p):
    A = W.random_mmatrix(24, 0.3, 20 + seed)
    Ls, U = orc.ilut(A, tau, p)
    Lb, Ub = _dense_ilut(dense(A), tau, p)
    np.testing.assert_allclose(unit_lower(Ls), Lb, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(dense(U), Ub, rtol=1e-12, atol=1e-14)
    assert np.all(np.diff(Ls.row_ptr) <= p)
    assert np.all(np.diff(U.row_ptr) <= p + 1)


def test_ilut_27pt_signs_and_counts(orc):
    """On the 27-point anisotropic M-matrix: row counts <= p per part, positive
    pivots, nonpositive off-diagonal factor entries (M-matrix sign pattern)."""
    A = W.aniso27(10)
    Ls, U = orc.ilut(A, 1e-3, 20)
    assert np.all(np.diff(Ls.row_ptr) <= 20)
    assert np.all(np.diff(U.row_ptr) <= 21)
    d, dinv, Us = orc.scale_rows(U)
    assert np.all(d > 0)
    assert np.all(Ls.val <= 0) and np.all(Us.val <= 0)
    # the drop rule removes the weak in-plane couplings of the strongly
    # z-anisotropic operator but keeps the z-couplings
    assert Ls.nnz > 0


# --------------------------------------------------------------------------
# row scaling (eqs. extractD, newD)
# --------------------------------------------------------------------------

def test_scale_rows_definition(orc):
    A = W.vardens7(6)
    Ls, U = orc.iluk(A, 1)
    d, dinv, Us = orc.scale_rows(U)
    Ud = dense(U)
    np.testing.assert_array_equal(d, np.diag(Ud))
    np.testing.assert_array_equal(dinv, 1.0 / np.diag(Ud))
    Ut = np.eye(A.n) + dense(Us)
    # D U~ = U: diag(U~) = 1 exactly and every scaled entry is one IEEE division
    rows = np.repeat(np.arange(U.n), np.diff(U.row_ptr))
    off = U.col != rows
    np.testing.assert_array_equal(Us.val, U.val[off] / d[rows[off]])
    np.testing.assert_allclose(np.diag(d) @ Ut, Ud, rtol=1e-15, atol=0)
    assert np.all(np.diag(Ut) == 1.0)


def test_scale_rows_zero_pivot_reported(orc):
    U = W.CSR.from_dense(np.array([[2.0, 1.0, 0.0], [0.0, 1.0, 3.0], [0.0, 0.0, 1.0]]))
    U.val[U.row_ptr[1]] = 0.0  # u_11 = 0 but still stored
    with pytest.raises(orc.OracleError) as e:
        orc.scale_rows(U)
    assert e.value.code == 1 and e.value.row == 1


def test_scaling_reduces_departure_from_normality(orc):
    """Section 5.1, Table 1: for the ill-conditioned variable-density operator
    dep(U) is orders of magnitude above dep(D^{-1}U), which equals dep(L)."""
    A = W.vardens7(8)
    Ls, U = orc.ilu0(A)
    d, dinv, Us = orc.scale_rows(U)
    depU = orc.dep_triangular(U)
    depUs = orc.dep_triangular(Us)
    depL = orc.dep_triangular(Ls)
    assert depU > 100 * depUs
    assert depUs == pytest.approx(depL, rel=1e-12)
