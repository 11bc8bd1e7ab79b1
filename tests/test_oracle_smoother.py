"""Pins for the oracle's smoother path: substitution, Richardson / Neumann
series, level sets, departure from normality, the smoother step, the mixed
form and outer convergence (CPU only)."""
import os

import numpy as np
import pytest
import scipy.linalg as sla

from paper_2111_09512_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense(M):
    return M.to_dense()


def factors(orc, A, kind="ilu0", **kw):
    if kind == "ilu0":
        Ls, U = orc.ilu0(A)
    elif kind == "iluk":
        Ls, U = orc.iluk(A, kw["k"])
    else:
        Ls, U = orc.ilut(A, kw["tau"], kw["p"])
    d, dinv, Us = orc.scale_rows(U)
    return Ls, U, d, dinv, Us


# --------------------------------------------------------------------------
# direct triangular solves (Section 4)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("uplo", ["L", "U"])
@pytest.mark.parametrize("unit", [True, False])
def test_trisolve_matches_scipy(orc, uplo, unit):
    rng = np.random.default_rng(5)
    n = 50
    T = np.where(rng.random((n, n)) < 0.2, rng.uniform(-1, 1, (n, n)), 0.0)
    T = np.tril(T, -1) if uplo == "L" else np.triu(T, 1)
    np.fill_diagonal(T, rng.uniform(1, 2, n))
    b = rng.uniform(-1, 1, n)
    Tc = W.CSR.from_dense(T)
    x = orc.trisolve(Tc, uplo, unit, b)
    Tref = T.copy()
    if unit:
        np.fill_diagonal(Tref, 1.0)
    ref = sla.solve_triangular(Tref, b, lower=(uplo == "L"))
    np.testing.assert_allclose(x, ref, rtol=1e-12, atol=1e-13)


def test_trisolve_rejects_wrong_side_and_zero_pivot(orc):
    T = W.CSR.from_dense(np.array([[1.0, 2.0], [0.0, 1.0]]))
    with pytest.raises(orc.OracleError):
        orc.trisolve(T, "L", True, np.ones(2))
    T = W.CSR.from_dense(np.array([[1.0, 0.0], [3.0, 0.0]]))
    T.val[:] = [1.0, 3.0]
    with pytest.raises(orc.OracleError):  # row 1 has no stored diagonal
        orc.trisolve(T, "L", False, np.ones(2))


# --------------------------------------------------------------------------
# Richardson = truncated Neumann series (eqs. richard, Neumann, Neuman)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("m", [1, 2, 3, 5, 8])
def test_richardson_is_truncated_neumann_series(orc, m):
    A = W.vardens7(5)
    Ls, U, d, dinv, Us = factors(orc, A, "iluk", k=1)
    rhs = W.rhs(A.n, 3)
    for N in (Ls, Us):
        Nd = dense(N)
        ref = np.zeros(A.n)
        term = rhs.copy()
        for _ in range(m):
            ref += term
            term = -Nd @ term
        got = orc.richardson(N, rhs, m)
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_richardson_level_exactness_and_nilpotence(orc):
    """After k steps every row whose level is < k holds its final value, bit for
    bit (same row summation order as substitution); m >= depth(N) reproduces the
    substitution exactly because N is nilpotent (end of Section 5.2)."""
    A = W.aniso27(6)
    Ls, U, d, dinv, Us = factors(orc, A, "ilut", tau=1e-3, p=20)
    rhs = W.rhs(A.n, 4)
    for N, uplo in ((Ls, "L"), (Us, "U")):
        lev, depth = orc.levels(N, uplo)
        exact = orc.trisolve(N, uplo, True, rhs)
        for k in (1, 2, 5, depth // 2, depth):
            yk = orc.richardson(N, rhs, k)
            done = lev < k
            assert np.array_equal(yk[done], exact[done])
        assert np.array_equal(orc.richardson(N, rhs, depth + 3), exact)


def test_unscaled_jacobi_equals_scaled_richardson(orc):
    """Jacobi on U z = y (eq. LUiterMat, G_U = I - D_U^{-1} U) is the Richardson
    iteration on the row-scaled factor: z_{k+1} = D^{-1} y - U~_s z_k (eq.
    richard).  Dense Jacobi vs the oracle's scaled Richardson."""
    A = W.vardens7(5)
    Ls, U, d, dinv, Us = factors(orc, A, "ilu0")
    y = W.rhs(A.n, 1)
    Ud = dense(U)
    D = np.diag(Ud)
    z = np.zeros(A.n)
    for m in range(1, 7):
        z = (y - (Ud - np.diag(D)) @ z) / D
        got = orc.richardson(Us, dinv * y, m)
        np.testing.assert_allclose(got, z, rtol=1e-12, atol=1e-12 * np.abs(z).max())


# --------------------------------------------------------------------------
# level sets (Section 4)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("N", [3, 4, 6, 9])
def test_level_depth_closed_forms(orc, N):
    """Every lower neighbour decreases phi by at least 1 and interior points
    have a neighbour at phi - 1, so the DAG depth is phi_max + 1:
    7-pt ILU(0): phi = x+y+z, depth 3(N-1)+1 (and level = x+y+z exactly);
    7-pt ILU(1): phi = x+2y+3z, depth 6(N-1)+1;
    27-pt ILU(0): phi = x+2y+4z, depth 7(N-1)+1.  The U factor mirrors L."""
    A = W.poisson7(N)
    Ls, U = orc.ilu0(A)
    lev, depth = orc.levels(Ls, "L")
    assert depth == 3 * (N - 1) + 1
    i = np.arange(A.n)
    np.testing.assert_array_equal(lev, i % N + (i // N) % N + i // (N * N))
    assert orc.levels(U, "U")[1] == depth
    Ls1, U1 = orc.iluk(W.vardens7(N), 1)
    assert orc.levels(Ls1, "L")[1] == 6 * (N - 1) + 1
    assert orc.levels(U1, "U")[1] == 6 * (N - 1) + 1
    Ls27, U27 = orc.ilu0(W.aniso27(N))
    assert orc.levels(Ls27, "L")[1] == 7 * (N - 1) + 1


def test_levels_are_a_valid_schedule(orc):
    A = W.permuted_longrange7(6, seed=1)
    Ls, U = orc.ilu0(A)
    for T, uplo in ((Ls, "L"), (U, "U")):
        lev, depth = orc.levels(T, uplo)
        rows = np.repeat(np.arange(T.n), np.diff(T.row_ptr))
        off = T.col != rows
        assert np.all(lev[rows[off]] > lev[T.col[off]])
        assert lev.max() + 1 == depth


# --------------------------------------------------------------------------
# departure from normality (eq. depB, eq. diagDep)
# --------------------------------------------------------------------------

def test_dep_closed_form_vs_eigenvalues(orc):
    rng = np.random.default_rng(9)
    for n in (5, 12):
        T = np.triu(rng.uniform(-1, 1, (n, n)))
        lam = np.linalg.eigvals(T)
        dep_def = np.sqrt(np.linalg.norm(T, "fro") ** 2 - np.sum(np.abs(lam) ** 2))
        assert orc.dep_triangular(W.CSR.from_dense(T)) == pytest.approx(dep_def, rel=1e-8)
    Dg = W.CSR.from_dense(np.diag(rng.uniform(1, 2, 7)))
    assert orc.dep_triangular(Dg) == 0.0  # eq. diagDep: a normal (diagonal) factor


def test_dep_before_and_after_scaling_dense(orc):
    """dep before and after row scaling, closed form vs eigenvalues of the dense factor."""
    A = W.vardens7(4)
    Ls, U, d, dinv, Us = factors(orc, A, "ilu0")
    for T, Td in ((U, dense(U)), (Us, np.eye(A.n) + dense(Us))):
        lam = np.linalg.eigvals(Td)
        dep_def = np.sqrt(max(np.linalg.norm(Td, "fro") ** 2 - np.sum(np.abs(lam) ** 2), 0.0))
        assert orc.dep_triangular(T) == pytest.approx(dep_def, rel=1e-6)


def test_table1_golden_identity():
    """Table 1 (Section 5.1) prints dep(D^{-1}U) equal to dep(L) in every row;
    the symmetric-A identity U~ = L^T (tested on the oracle above) explains it."""
    rows = []
    with open(os.path.join(GOLDEN, "table1_dep.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, dim, depL, depU, depDU, depRC = line.split()
            rows.append((name, int(dim), float(depL), float(depU), float(depDU), float(depRC)))
    assert len(rows) == 8
    for name, dim, depL, depU, depDU, depRC in rows:
        assert depDU == depL, name
        assert depU > 10 * depDU, name


# --------------------------------------------------------------------------
# the smoother step (eq. ILUsplit; Algorithm 2)
# --------------------------------------------------------------------------

def _dense_smoother_matrix(Ls, Us, dinv, mL, mU):
    n = Ls.n
    def neumann(N, m):
        S = np.zeros((n, n))
        T = np.eye(n)
        for _ in range(m):
            S += T
            T = -N @ T
        return S
    return neumann(dense(Us), mU) @ np.diag(dinv) @ neumann(dense(Ls), mL)


@pytest.mark.parametrize("mL,mU,outer", [(1, 1, 1), (3, 3, 1), (2, 5, 2), (4, 4, 3)])
def test_smoother_equals_dense_formula(orc, mL, mU, outer):
    """x_{k+1} = x_k + M_m (b - A x_k) with M_m the product of the truncated
    Neumann series (dense, from eqs. ILUsplit and Neumann)."""
    A = W.vardens7(5)
    Ls, U, d, dinv, Us = factors(orc, A, "iluk", k=1)
    b = W.rhs(A.n, 0)
    x0 = W.rhs(A.n, 11)
    Mm = _dense_smoother_matrix(Ls, Us, dinv, mL, mU)
    Ad = dense(A)
    x = x0.copy()
    for _ in range(outer):
        x = x + Mm @ (b - Ad @ x)
    got = orc.smooth(A, Ls, Us, dinv, b, x0, outer, mL, mU)
    np.testing.assert_allclose(got, x, rtol=1e-11, atol=1e-11 * np.abs(x).max())


def test_smoother_m1_closed_form(orc):
    """m_L = m_U = 1 reduces the smoother to x + D^{-1}(b - A x), D = diag(U)."""
    A = W.poisson7(6)
    Ls, U, d, dinv, Us = factors(orc, A, "ilu0")
    b = W.rhs(A.n, 0)
    x0 = W.rhs(A.n, 2)
    got = orc.smooth(A, Ls, Us, dinv, b, x0, 1, 1, 1)
    ref = x0 + dinv * (b - dense(A) @ x0)
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-14)


def test_smoother_exact_on_tridiagonal(orc):
    """Tridiagonal A: ILU(0) is the exact LU, so one direct smoothing step from
    any x0 solves A x = b; with m >= n Richardson steps the iteration is exact too."""
    n = 40
    A = W.tridiag(n)
    Ls, U, d, dinv, Us = factors(orc, A, "ilu0")
    b = W.rhs(n, 0)
    ref = np.linalg.solve(dense(A), b)
    x0 = W.rhs(n, 5)
    xd = orc.smooth(A, Ls, Us, dinv, b, x0, 1, 1, 1, direct=True)
    np.testing.assert_allclose(xd, ref, rtol=1e-12, atol=1e-12)
    xi = orc.smooth(A, Ls, Us, dinv, b, x0, 1, n, n)
    np.testing.assert_allclose(xi, ref, rtol=1e-12, atol=1e-12)


def test_smoother_is_affine(orc):
    """S(b, x0) = S(b, 0) + S(0, x0): the step is x0 + M(b - A x0)."""
    A = W.aniso27(5)
    Ls, U, d, dinv, Us = factors(orc, A, "ilut", tau=1e-3, p=20)
    b = W.rhs(A.n, 0)
    x0 = W.rhs(A.n, 1)
    z = np.zeros(A.n)
    lhs = orc.smooth(A, Ls, Us, dinv, b, x0, 1, 4, 4)
    rhs_ = orc.smooth(A, Ls, Us, dinv, b, z, 1, 4, 4) + orc.smooth(A, Ls, Us, dinv, z, x0, 1, 4, 4)
    np.testing.assert_allclose(lhs, rhs_, rtol=1e-12, atol=1e-12 * np.abs(lhs).max())


def test_direct_mode_equals_ldu_solve(orc):
    A = W.vardens7(5)
    Ls, U, d, dinv, Us = factors(orc, A, "iluk", k=1)
    b = W.rhs(A.n, 0)
    x = orc.smooth(A, Ls, Us, dinv, b, np.zeros(A.n), 1, 0, 0, direct=True)
    M = (np.eye(A.n) + dense(Ls)) @ dense(U)
    np.testing.assert_allclose(x, np.linalg.solve(M, b), rtol=1e-10, atol=1e-12)


def test_unscaled_variant_formula_and_failure(orc):
    """Unscaled Richardson z_k = y - (U - I) z_{k-1} (Section 6.1: the
    iterative solves fail unless scaled): dense check, and on the
    variable-density operator it blows up while the scaled form does not."""
    A = W.vardens7(5)
    Ls, U, d, dinv, Us = factors(orc, A, "ilu0")
    b = W.rhs(A.n, 0)
    x = orc.smooth_unscaled(A, Ls, U, b, np.zeros(A.n), 1, 3, 3)
    Ud = dense(U)
    Nu = Ud - np.eye(A.n)
    r = b.copy()
    y = np.zeros(A.n)
    for _ in range(3):
        y = r - dense(Ls) @ y
    z = np.zeros(A.n)
    for _ in range(3):
        z = y - Nu @ z
    np.testing.assert_allclose(x, z, rtol=1e-12, atol=1e-12 * np.abs(z).max())
    xs = orc.smooth(A, Ls, Us, dinv, b, np.zeros(A.n), 1, 3, 3)
    ref = np.linalg.solve(dense(A), b)
    err_s = np.linalg.norm(xs - ref) / np.linalg.norm(ref)
    err_u = np.linalg.norm(x - ref) / np.linalg.norm(ref)
    assert err_s < 1.0 < err_u


# --------------------------------------------------------------------------
# mixed-precision emulation and outer convergence
# --------------------------------------------------------------------------

def test_mixed_m1_closed_form(orc):
    """With one Richardson step per factor the mixed form is
    x + (double)(float)(dinv * (double)(float)(b - A x))."""
    A = W.poisson7(6)
    Ls, U, d, dinv, Us = factors(orc, A, "ilu0")
    b = W.rhs(A.n, 0)
    x0 = W.rhs(A.n, 2)
    r = orc.residual(A, b, x0)
    s = (dinv * r.astype(np.float32).astype(np.float64)).astype(np.float32)
    ref = x0 + s.astype(np.float64)
    got = orc.smooth_mixed(A, Ls, Us, dinv, b, x0, 1, 1, 1)
    np.testing.assert_array_equal(got, ref)


def _mixed_by_scalars(A, Ls, Us, dinv, b, x0, outer, mL, mU):
    """The FP32-inner smoother (reading 11's rounding points) written with
    numpy scalars, one operation at a time: the residual summed in FP64 in
    ascending column order; the Richardson loops on np.float32 values and
    iterates, each row's products accumulated in np.float32 in ascending
    column order from +0; s = fp32(dinv * y) in FP64; x += fp64(z)."""
    f32 = np.float32

    def rows(M):
        return [(M.col[M.row_ptr[i]:M.row_ptr[i + 1]], M.val[M.row_ptr[i]:M.row_ptr[i + 1]]) for i in range(M.n)]

    Ar, Lr, Ur = rows(A), rows(Ls), rows(Us)
    Lr32 = [(c, [f32(v) for v in vals]) for c, vals in Lr]
    Ur32 = [(c, [f32(v) for v in vals]) for c, vals in Ur]

    def richardson32(R, rhs, m):
        y = [f32(0.0)] * len(rhs)
        for _ in range(m):
            new = []
            for i, (cols, vals) in enumerate(R):
                t = f32(0.0)
                for j, v in zip(cols, vals):
                    t = f32(t + f32(v * y[j]))
                new.append(f32(rhs[i] - t))
            y = new
        return y

    x = [float(v) for v in x0]
    for _ in range(outer):
        r = []
        for i, (cols, vals) in enumerate(Ar):
            t = 0.0
            for j, v in zip(cols, vals):
                t = t + float(v) * x[j]
            r.append(f32(float(b[i]) - t))
        y = richardson32(Lr32, r, mL)
        s = [f32(float(dinv[i]) * float(y[i])) for i in range(len(y))]
        z = richardson32(Ur32, s, mU)
        x = [x[i] + float(z[i]) for i in range(len(x))]
    return np.array(x)


@pytest.mark.parametrize("mL,mU", [(2, 2), (3, 3), (2, 3)])
def test_mixed_fp32_loop_by_scalars(orc, mL, mU):
    """The FP32 loop of the mixed emulation, re-derived with np.float32 scalar
    arithmetic on a small ILUT case (many entries per row, so the order and
    the precision of each row's accumulation decide the last bits): bit for
    bit, over two outer steps from a nonzero guess.  Also differs from the
    FP64 smoother, so the FP32 rounding really happens."""
    A = W.aniso27(4)
    Ls, U, d, dinv, Us = factors(orc, A, "ilut", tau=1e-3, p=20)
    b = W.rhs(A.n, 0)
    x0 = W.rhs(A.n, 2)
    got = orc.smooth_mixed(A, Ls, Us, dinv, b, x0, 2, mL, mU)
    want = _mixed_by_scalars(A, Ls, Us, dinv, b, x0, 2, mL, mU)
    np.testing.assert_array_equal(got, want)
    assert not np.array_equal(got, orc.smooth(A, Ls, Us, dinv, b, x0, 2, mL, mU))


def test_mixed_close_to_fp64(orc):
    A = W.aniso27(8)
    Ls, U, d, dinv, Us = factors(orc, A, "ilut", tau=1e-3, p=20)
    b = W.rhs(A.n, 0)
    x64 = orc.smooth(A, Ls, Us, dinv, b, np.zeros(A.n), 2, 4, 4)
    x32 = orc.smooth_mixed(A, Ls, Us, dinv, b, np.zeros(A.n), 2, 4, 4)
    rel = np.linalg.norm(x32 - x64) / np.linalg.norm(x64)
    assert 0 < rel < 1e-5


def test_outer_convergence_to_solution(orc):
    """Repeated smoothing (ILU as a regular splitting of an M-matrix) drives
    the relative residual (eq. relres) below 1e-8; the iterate then agrees with
    a dense solve.  The mixed form reaches the tolerance in the same number of
    outer steps here."""
    A = W.poisson7(8)
    Ls, U, d, dinv, Us = factors(orc, A, "ilu0")
    b = W.rhs(A.n, 0)
    k, x, hist = orc.smooth_until(A, Ls, Us, dinv, b, np.zeros(A.n), 3, 3, 1e-8, 200)
    assert k <= 200 and hist[-1] < 1e-8 and np.all(np.diff(hist) < 0)
    ref = np.linalg.solve(dense(A), b)
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-7
    km, xm, histm = orc.smooth_until(A, Ls, Us, dinv, b, np.zeros(A.n), 3, 3, 1e-8, 200, mixed=True)
    assert km == k


def test_golden_regression_poisson8(orc):
    """Oracle outputs written by tests/golden/make_golden.py (which calls only
    the oracle).  Guards against unintended changes to the oracle's arithmetic."""
    import json

    with open(os.path.join(GOLDEN, "oracle_poisson8.json")) as f:
        g = json.load(f)
    A = W.poisson7(8)
    Ls, U, d, dinv, Us = factors(orc, A, "ilu0")
    b = W.rhs(A.n, 0)
    x = orc.smooth(A, Ls, Us, dinv, b, np.zeros(A.n), 1, 3, 3)
    assert [float(v) for v in x[g["idx"]]] == g["x_at_idx"]
    assert float(orc.nrm2(x)) == g["nrm2"]


@pytest.mark.parametrize("N,kind", [(9, "ilu0"), (7, "ilut")])
def test_smooth_omp_equals_sequential(orc, N, kind):
    """The row-parallel variant used for the CPU baseline sums every row in the
    same order as the sequential smoother, so the two agree bit for bit."""
    A = W.poisson7(N) if kind == "ilu0" else W.aniso27(N)
    Ls, U, d, dinv, Us = factors(orc, A, kind, tau=1e-3, p=20)
    b, x0 = W.rhs(A.n, 0), W.rhs(A.n, 3)
    assert orc.omp_threads() >= 1
    for outer, mL, mU in ((1, 1, 1), (2, 4, 4), (1, 3, 2)):
        np.testing.assert_array_equal(orc.smooth_omp(A, Ls, Us, dinv, b, x0, outer, mL, mU),
                                      orc.smooth(A, Ls, Us, dinv, b, x0, outer, mL, mU))
