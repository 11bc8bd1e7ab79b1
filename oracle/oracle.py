"""ctypes wrapper over the plain-C FP64 oracle (``oracle.c``).

TEST INFRASTRUCTURE.  Only the tests, the package smoke check and the
benchmark's CPU-baseline leg use it.  It imports nothing from the GPU package;
its inputs are numpy CSR triples (``row_ptr`` int32, ``col`` int32, ``val``
float64) such as the seeded generators produce.

Every function names the passage of arXiv 2111.09512 it follows; the C file
carries the full statement of each step.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB points the wrapper at another build of oracle.c (the sanitizer build of the tests)
_LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")


class _OrcCSR(C.Structure):
    _fields_ = [
        ("n", C.c_int),
        ("nnz", C.c_longlong),
        ("rp", C.POINTER(C.c_int)),
        ("col", C.POINTER(C.c_int)),
        ("val", C.POINTER(C.c_double)),
    ]


class OracleError(RuntimeError):
    def __init__(self, code: int, row: int, what: str):
        names = {1: "zero pivot", 2: "out of memory", 3: "pattern error"}
        super().__init__(f"oracle {what}: {names.get(code, code)} at row {row}")
        self.code = code
        self.row = row


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b

            _b.build()
        _lib = C.CDLL(_LIB_PATH)
        L = _lib
        L.orc_csr_free.argtypes = [C.POINTER(_OrcCSR)]
        L.orc_iluk.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_int, C.POINTER(_OrcCSR), C.POINTER(_OrcCSR),
                               C.POINTER(C.c_int)]
        L.orc_ilut.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_double, C.c_int, C.POINTER(_OrcCSR),
                               C.POINTER(_OrcCSR), C.POINTER(C.c_int)]
        L.orc_scale_rows.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, _f64p, _i32p, _i32p, _f64p,
                                     C.POINTER(C.c_int)]
        L.orc_scale_rowcol.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_int, _f64p, _f64p, _f64p, _i32p, _i32p,
                                       _f64p, C.POINTER(C.c_int)]
        L.orc_smooth_rowcol.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p,
                                        _f64p, _f64p, _f64p, _f64p, C.c_int, C.c_int, C.c_int, C.c_int, _f64p,
                                        _f32p]
        L.orc_smooth_rowcol.restype = None
        L.orc_gs_split.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p, _f64p, C.POINTER(C.c_int)]
        L.orc_gs_smooth.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p, _f64p, _f64p, _f64p,
                                    C.c_int, C.c_int, C.c_int, _f64p, _f32p]
        L.orc_gs_smooth.restype = None
        L.orc_fgmres.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p, _f64p,
                                 C.c_int, C.c_int, C.c_int, _f64p, _f64p, C.c_int, C.c_int, C.c_double, C.c_double,
                                 _f64p, _f64p]
        L.orc_ilu0_fixed_point.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_int, _f64p, _f64p]
        L.orc_spmv.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, _f64p]
        L.orc_spmv.restype = None
        L.orc_residual.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, _f64p, _f64p]
        L.orc_residual.restype = None
        L.orc_richardson.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p, C.c_int, _f64p, _f64p]
        L.orc_richardson.restype = None
        L.orc_trisolve.argtypes = [C.c_int, _i32p, _i32p, _f64p, C.c_int, C.c_int, _f64p, _f64p,
                                   C.POINTER(C.c_int)]
        L.orc_smooth.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p, _f64p,
                                 _f64p, _f64p, C.c_int, C.c_int, C.c_int, C.c_int, _f64p]
        L.orc_smooth.restype = None
        L.orc_smooth_omp.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p,
                                     _f64p, _f64p, _f64p, C.c_int, C.c_int, C.c_int, _f64p]
        L.orc_smooth_omp.restype = None
        L.orc_omp_threads.argtypes = []
        L.orc_omp_threads.restype = C.c_int
        L.orc_unit_shift.argtypes = [C.c_int, _i32p, _i32p, _f64p, _f64p]
        L.orc_unit_shift.restype = None
        L.orc_smooth_unscaled.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p, _i32p, _i32p,
                                          _f64p, _f64p, _f64p, C.c_int, C.c_int, C.c_int, _f64p]
        L.orc_smooth_unscaled.restype = None
        L.orc_smooth_mixed.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p,
                                       _f64p, _f64p, _f64p, C.c_int, C.c_int, C.c_int, _f64p, _f32p]
        L.orc_smooth_mixed.restype = None
        L.orc_nrm2.argtypes = [C.c_int, _f64p]
        L.orc_nrm2.restype = C.c_double
        L.orc_smooth_until.argtypes = [C.c_int, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p,
                                       _f64p, _f64p, _f64p, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int,
                                       _f64p, _f64p, _f32p]
        L.orc_levels.argtypes = [C.c_int, _i32p, _i32p, C.c_int, _i32p]
        L.orc_dep_triangular.argtypes = [C.c_int, _i32p, _i32p, _f64p]
        L.orc_dep_triangular.restype = C.c_double
    return _lib


# --------------------------------------------------------------------------
# plain containers
# --------------------------------------------------------------------------

class Mat:
    """Host CSR triple (row_ptr int32, col int32, val float64)."""

    def __init__(self, n, row_ptr, col, val):
        self.n = int(n)
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)

    @property
    def nnz(self):
        return int(self.row_ptr[-1])

    def to_dense(self):
        d = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        d[rows, self.col] = self.val
        return d


def _mat(A) -> Mat:
    if isinstance(A, Mat):
        return A
    return Mat(A.n, A.row_ptr, A.col, A.val)


def _take(m: _OrcCSR) -> Mat:
    n = m.n
    rp = np.ctypeslib.as_array(m.rp, shape=(n + 1,)).copy()
    nnz = int(m.nnz)
    if nnz:
        col = np.ctypeslib.as_array(m.col, shape=(nnz,)).copy()
        val = np.ctypeslib.as_array(m.val, shape=(nnz,)).copy()
    else:
        col = np.zeros(0, np.int32)
        val = np.zeros(0, np.float64)
    lib().orc_csr_free(C.byref(m))
    return Mat(n, rp, col, val)


# --------------------------------------------------------------------------
# factorizations
# --------------------------------------------------------------------------

def iluk(A, k: int):
    """ILU(k) (Section 1, Saad's level-of-fill ILU; Section 3.1 symbolic/numeric split).
    Returns (Ls strictly lower, U upper with diagonal first)."""
    A = _mat(A)
    Lm, Um, bad = _OrcCSR(), _OrcCSR(), C.c_int(-1)
    st = lib().orc_iluk(A.n, A.row_ptr, A.col, A.val, int(k), C.byref(Lm), C.byref(Um), C.byref(bad))
    if st:
        raise OracleError(st, bad.value, f"ILU({k})")
    return _take(Lm), _take(Um)


def ilu0(A):
    """ILU(0): zero fill on the pattern of A (Table 1's 'nofill')."""
    return iluk(A, 0)


def ilut(A, tau: float, p: int):
    """ILUT(tau, p), dual-threshold ILU in A's units (Sections 4.2, 6.1)."""
    A = _mat(A)
    Lm, Um, bad = _OrcCSR(), _OrcCSR(), C.c_int(-1)
    st = lib().orc_ilut(A.n, A.row_ptr, A.col, A.val, float(tau), int(p), C.byref(Lm), C.byref(Um),
                        C.byref(bad))
    if st:
        raise OracleError(st, bad.value, f"ILUT({tau},{p})")
    return _take(Lm), _take(Um)


def factor(A, kind: str, params: dict):
    if kind == "ilu0":
        return ilu0(A)
    if kind == "iluk":
        return iluk(A, params["k"])
    if kind == "ilut":
        return ilut(A, params["tau"], params["p"])
    raise KeyError(kind)


# --------------------------------------------------------------------------
# scaling and kernels of the smoother
# --------------------------------------------------------------------------

def scale_rows(U):
    """Row scaling D = diag(U), U~ = D^{-1} U (Section 5.1, eqs. extractD, newD).
    Returns (d, dinv, Us) with Us the strictly upper part of U~."""
    U = _mat(U)
    n = U.n
    nnz = U.nnz - n
    d = np.empty(n)
    dinv = np.empty(n)
    rp = np.empty(n + 1, np.int32)
    col = np.empty(max(nnz, 0), np.int32)
    val = np.empty(max(nnz, 0))
    bad = C.c_int(-1)
    st = lib().orc_scale_rows(n, U.row_ptr, U.col, U.val, d, dinv, rp, col, val, C.byref(bad))
    if st:
        raise OracleError(st, bad.value, "row scaling")
    return d, dinv, Mat(n, rp, col, val)


def scale_rowcol(U, iters: int = 5):
    """Row/column scaling U^ = D_r U D_c with a unit diagonal (Section 5.1, eq.
    rowcolScale; Ruiz steps in the max norm, then d_r,i = 1/(u_ii d_c,i)).
    Returns (dr, dc, Us_hat, dr_before_unit_diagonal)."""
    U = _mat(U)
    n = U.n
    nnz = U.nnz - n
    dr = np.empty(n)
    dc = np.empty(n)
    drr = np.empty(n)
    rp = np.empty(n + 1, np.int32)
    col = np.empty(max(nnz, 0), np.int32)
    val = np.empty(max(nnz, 0))
    bad = C.c_int(-1)
    st = lib().orc_scale_rowcol(n, U.row_ptr, U.col, U.val, int(iters), dr, dc, drr, rp, col, val, C.byref(bad))
    if st:
        raise OracleError(st, bad.value, "row/column scaling")
    return dr, dc, Mat(n, rp, col, val), drr


def smooth_rowcol(A, Ls, Us_hat, dr, dc, b, x0, outer: int, mL: int, mU: int, mixed: bool = False,
                  direct: bool = False):
    """Smoother with the row/column-scaled U (eq. rowcolScale): s = d_r * y,
    m_U steps on U^ v = s, x += d_c * v.  mixed: FP32 Richardson loops;
    direct: both solves by substitution."""
    A, Ls, Us_hat = _mat(A), _mat(Ls), _mat(Us_hat)
    n = A.n
    x = np.array(x0, dtype=np.float64, copy=True)
    ws = np.empty(5 * n)
    fws = np.empty(4 * n, np.float32)
    mode = 2 if direct else (1 if mixed else 0)
    lib().orc_smooth_rowcol(n, A.row_ptr, A.col, A.val, Ls.row_ptr, Ls.col, Ls.val, Us_hat.row_ptr, Us_hat.col,
                            Us_hat.val, np.ascontiguousarray(dr, np.float64), np.ascontiguousarray(dc, np.float64),
                            np.ascontiguousarray(b, np.float64), x, int(outer), int(mL), int(mU), mode, ws, fws)
    return x


def gs_split(A):
    """Polynomial Gauss-Seidel set-up: (Gs = D^{-1} L strictly lower, dinv = 1/diag(A))."""
    A = _mat(A)
    n = A.n
    rp = np.empty(n + 1, np.int32)
    col = np.empty(max(A.nnz, 1), np.int32)
    val = np.empty(max(A.nnz, 1))
    dinv = np.empty(n)
    bad = C.c_int(-1)
    st = lib().orc_gs_split(n, A.row_ptr, A.col, A.val, rp, col, val, dinv, C.byref(bad))
    if st:
        raise OracleError(st, bad.value, "Gauss-Seidel split")
    nnz = int(rp[-1])
    return Mat(n, rp, col[:nnz].copy(), val[:nnz].copy()), dinv


def gs_smooth(A, Gs, dinv, b, x0, outer: int, m: int, mixed: bool = False):
    """Polynomial Gauss-Seidel smoother: x += sum_{j<m} (-D^{-1}L)^j D^{-1}(b - A x), `outer` times."""
    A, Gs = _mat(A), _mat(Gs)
    n = A.n
    x = np.array(x0, dtype=np.float64, copy=True)
    ws = np.empty(3 * n)
    fws = np.empty(3 * n, np.float32)
    lib().orc_gs_smooth(n, A.row_ptr, A.col, A.val, Gs.row_ptr, Gs.col, Gs.val, np.ascontiguousarray(dinv, np.float64),
                        np.ascontiguousarray(b, np.float64), x, int(outer), int(m), int(bool(mixed)), ws, fws)
    return x


def fgmres(A, Ls, Us, dinv, b, x0, m: int, max_iters: int, tol: float, outer: int = 1, mL: int = 3, mU: int = 3,
           norm_a: float = 0.0):
    """FGMRES(m) with the ILU smoother (outer steps x m_L/m_U from z = 0) as right
    preconditioner (Section 6).  Stops when the residual estimate over
    (||b|| + norm_a ||x||) drops below tol: norm_a = 0 is the relative residual
    of eq. relres, norm_a = ||A||_2 the norm-wise relative backward error of eq.
    nbre (the iterate is formed after every step for its norm).  Returns
    (steps, x, history of the estimates)."""
    if not norm_a >= 0.0:
        raise ValueError("norm_a must be >= 0")
    A, Ls, Us = _mat(A), _mat(Ls), _mat(Us)
    n = A.n
    x = np.array(x0, dtype=np.float64, copy=True)
    ws = np.empty((2 * m + 8) * n + (m + 1) * (m + 4))
    hist = np.zeros(max_iters + 1)
    k = lib().orc_fgmres(n, A.row_ptr, A.col, A.val, Ls.row_ptr, Ls.col, Ls.val, Us.row_ptr, Us.col, Us.val,
                         np.ascontiguousarray(dinv, np.float64), int(outer), int(mL), int(mU),
                         np.ascontiguousarray(b, np.float64), x, int(m), int(max_iters), float(tol), float(norm_a),
                         hist, ws)
    return k, x, hist[: k + 1].copy()


def ilu0_fixed_point(A, sweeps: int):
    """ILU(0) by synchronous fixed-point sweeps (Section 7).  Returns (Ls, U, n_stable)
    where n_stable is the sweep after which the values stopped changing (sweeps + 1
    if they had not)."""
    A = _mat(A)
    n = A.n
    LU = np.empty(max(A.nnz, 1))
    ws = np.empty(A.nnz + n + 1)
    st = lib().orc_ilu0_fixed_point(n, A.row_ptr, A.col, A.val, int(sweeps), LU, ws)
    if st < 0:
        raise OracleError(3, -1, "fixed-point ILU(0)")
    rows = np.repeat(np.arange(n), np.diff(A.row_ptr))
    low = A.col < rows
    Lrp = np.concatenate([[0], np.cumsum(np.bincount(rows[low], minlength=n))]).astype(np.int32)
    Urp = np.concatenate([[0], np.cumsum(np.bincount(rows[~low], minlength=n))]).astype(np.int32)
    Ls = Mat(n, Lrp, A.col[low].copy(), LU[: A.nnz][low].copy())
    U = Mat(n, Urp, A.col[~low].copy(), LU[: A.nnz][~low].copy())
    return Ls, U, st


def spmv(N, x):
    N = _mat(N)
    y = np.empty(N.n)
    lib().orc_spmv(N.n, N.row_ptr, N.col, N.val, np.ascontiguousarray(x, np.float64), y)
    return y


def residual(A, b, x):
    """r = b - A x (eq. ILUsplit)."""
    A = _mat(A)
    r = np.empty(A.n)
    lib().orc_residual(A.n, A.row_ptr, A.col, A.val, np.ascontiguousarray(b, np.float64),
                       np.ascontiguousarray(x, np.float64), r)
    return r


def richardson(N, rhs, m: int):
    """m Richardson steps y_k = rhs - N y_{k-1} from y_0 = 0 (eq. richard; Algorithm 2)."""
    N = _mat(N)
    y = np.empty(N.n)
    tmp = np.empty(N.n)
    lib().orc_richardson(N.n, N.row_ptr, N.col, N.val, np.ascontiguousarray(rhs, np.float64), int(m), y, tmp)
    return y


def trisolve(T, uplo: str, unit: bool, rhs):
    """Direct triangular solve by substitution (Section 4)."""
    T = _mat(T)
    out = np.empty(T.n)
    bad = C.c_int(-1)
    st = lib().orc_trisolve(T.n, T.row_ptr, T.col, T.val, 0 if uplo == "L" else 1, 1 if unit else 0,
                            np.ascontiguousarray(rhs, np.float64), out, C.byref(bad))
    if st:
        raise OracleError(st, bad.value, "trisolve")
    return out


def smooth(A, Ls, Us, dinv, b, x0, outer: int, mL: int, mU: int, direct: bool = False):
    """The scaled ILU smoother, `outer` steps of x += U~^{-1} D^{-1} L^{-1}(b - A x) with
    the triangular solves replaced by mL / mU Richardson steps (Algorithm 2, eq. ILUsplit)."""
    A, Ls, Us = _mat(A), _mat(Ls), _mat(Us)
    n = A.n
    x = np.array(x0, dtype=np.float64, copy=True)
    ws = np.empty(5 * n)
    lib().orc_smooth(n, A.row_ptr, A.col, A.val, Ls.row_ptr, Ls.col, Ls.val, Us.row_ptr, Us.col, Us.val,
                     np.ascontiguousarray(dinv, np.float64), np.ascontiguousarray(b, np.float64), x,
                     int(outer), int(mL), int(mU), 1 if direct else 0, ws)
    return x


def smooth_omp(A, Ls, Us, dinv, b, x0, outer: int, mL: int, mU: int):
    """`smooth` (iterative form) with its row loops split among OpenMP threads;
    bit-identical to `smooth`.  For timing the CPU baseline on all host cores."""
    A, Ls, Us = _mat(A), _mat(Ls), _mat(Us)
    n = A.n
    x = np.array(x0, dtype=np.float64, copy=True)
    ws = np.empty(5 * n)
    lib().orc_smooth_omp(n, A.row_ptr, A.col, A.val, Ls.row_ptr, Ls.col, Ls.val, Us.row_ptr, Us.col, Us.val,
                         np.ascontiguousarray(dinv, np.float64), np.ascontiguousarray(b, np.float64), x,
                         int(outer), int(mL), int(mU), ws)
    return x


def omp_threads():
    """Threads `smooth_omp` runs on (OMP_NUM_THREADS, else every host thread)."""
    return int(lib().orc_omp_threads())


def unit_shift(U):
    """N = U - I (diagonal stored as u_ii - 1), the iteration matrix of unscaled Richardson."""
    U = _mat(U)
    Nv = np.empty(U.nnz)
    lib().orc_unit_shift(U.n, U.row_ptr, U.col, U.val, Nv)
    return Mat(U.n, U.row_ptr, U.col, Nv)


def smooth_unscaled(A, Ls, U, b, x0, outer: int, mL: int, mU: int):
    """Unscaled variant (Section 6.1: fails without scaling): z_k = y - (U - I) z_{k-1}."""
    A, Ls = _mat(A), _mat(Ls)
    Nm = unit_shift(U)
    n = A.n
    x = np.array(x0, dtype=np.float64, copy=True)
    ws = np.empty(5 * n)
    lib().orc_smooth_unscaled(n, A.row_ptr, A.col, A.val, Ls.row_ptr, Ls.col, Ls.val, Nm.row_ptr, Nm.col,
                              Nm.val, np.ascontiguousarray(b, np.float64), x, int(outer), int(mL), int(mU), ws)
    return x


def smooth_mixed(A, Ls, Us, dinv, b, x0, outer: int, mL: int, mU: int):
    """FP32-inner emulation: FP32 factor values, iterates and accumulation; FP64 residual,
    diagonal scaling and update of x."""
    A, Ls, Us = _mat(A), _mat(Ls), _mat(Us)
    n = A.n
    x = np.array(x0, dtype=np.float64, copy=True)
    ws = np.empty(2 * n)
    fws = np.empty(4 * n, np.float32)
    lib().orc_smooth_mixed(n, A.row_ptr, A.col, A.val, Ls.row_ptr, Ls.col, Ls.val, Us.row_ptr, Us.col, Us.val,
                           np.ascontiguousarray(dinv, np.float64), np.ascontiguousarray(b, np.float64), x,
                           int(outer), int(mL), int(mU), ws, fws)
    return x


def smooth_until(A, Ls, Us, dinv, b, x0, mL: int, mU: int, tol: float, max_outer: int, mixed: bool = False):
    """Outer steps until ||b - A x||_2 / ||b||_2 < tol (eq. relres).
    Returns (steps, x, history)."""
    A, Ls, Us = _mat(A), _mat(Ls), _mat(Us)
    n = A.n
    x = np.array(x0, dtype=np.float64, copy=True)
    hist = np.zeros(max_outer + 1)
    ws = np.empty(6 * n)
    fws = np.empty(4 * n, np.float32)
    k = lib().orc_smooth_until(n, A.row_ptr, A.col, A.val, Ls.row_ptr, Ls.col, Ls.val, Us.row_ptr, Us.col,
                               Us.val, np.ascontiguousarray(dinv, np.float64), np.ascontiguousarray(b, np.float64),
                               x, int(mL), int(mU), 1 if mixed else 0, float(tol), int(max_outer), hist, ws, fws)
    return k, x, hist[: min(k, max_outer) + 1]


def nrm2(v):
    return lib().orc_nrm2(len(v), np.ascontiguousarray(v, np.float64))


def levels(T, uplo: str):
    """Level sets of the elimination DAG (Section 4).  Returns (level per row, depth)."""
    T = _mat(T)
    lev = np.zeros(T.n, np.int32)
    depth = lib().orc_levels(T.n, T.row_ptr, T.col, 0 if uplo == "L" else 1, lev)
    if depth < 0:
        raise OracleError(3, -1, "levels")
    return lev, depth


def dep_triangular(T, unit_diag: bool = False):
    """Henrici departure from normality of a triangular matrix (eq. depB; eq. diagDep):
    ||T - diag(T)||_F.  ``unit_diag`` only documents that T's diagonal is implied."""
    T = _mat(T)
    return lib().orc_dep_triangular(T.n, T.row_ptr, T.col, T.val)
