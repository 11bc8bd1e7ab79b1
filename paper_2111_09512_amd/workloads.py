"""Seeded synthetic inputs for the scaled-ILU smoother.

This module only builds problem *inputs*: sparse operators A in CSR form,
right-hand sides b and initial guesses x0.  It holds none of the smoother's
arithmetic (no factorization, no scaling, no residual, no sweep, no solve), so
both the CPU oracle and the GPU path may take their inputs from it.

The paper measures on pressure matrices exported from PeleLM and Nalu-Wind and
on SuiteSparse matrices (Section 5.1, Tables 1-2; Section 6).  None of those is
available here; the generators below stand in for them with the character the
paper describes: symmetric, variable-coefficient, ill-conditioned pressure
operators with cut cells (Section 1), anisotropic and unstructured couplings
(Section 6.2).  Every random draw uses ``numpy.random.default_rng(seed)``.

Grid ordering is lexicographic, ``idx = x + N*y + N*N*z``.  Dirichlet
boundaries: a coupling to a point outside the grid is dropped and its weight
stays on the diagonal.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class CSR:
    """Square sparse matrix in CSR form, columns sorted ascending within a row."""

    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col: np.ndarray  # int32 [nnz]
    val: np.ndarray  # float64 [nnz]
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        d[rows, self.col] = self.val
        return d

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))

    @staticmethod
    def from_dense(d: np.ndarray) -> "CSR":
        d = np.asarray(d, dtype=np.float64)
        n = d.shape[0]
        mask = d != 0.0
        rp = np.zeros(n + 1, dtype=np.int32)
        rp[1:] = np.cumsum(mask.sum(1))
        rows, cols = np.nonzero(mask)
        return CSR(n, rp, cols.astype(np.int32), d[rows, cols].copy())

    def validate(self) -> None:
        """Structural checks: sizes, sorted unique columns, indices in range."""
        rp, col = self.row_ptr, self.col
        assert rp.dtype == np.int32 and col.dtype == np.int32 and self.val.dtype == np.float64
        assert rp.shape == (self.n + 1,) and rp[0] == 0
        assert np.all(np.diff(rp.astype(np.int64)) >= 0)
        assert col.shape == (self.nnz,) and self.val.shape == (self.nnz,)
        if self.nnz:
            assert col.min() >= 0 and col.max() < self.n
            # strictly increasing within each row
            d = np.diff(col.astype(np.int64))
            starts = rp[1:-1]
            inner = np.ones(self.nnz - 1, dtype=bool)
            inner[starts[(starts > 0) & (starts < self.nnz)] - 1] = False
            assert np.all(d[inner] > 0), "columns must be sorted and unique within a row"


# --------------------------------------------------------------------------
# structured-grid stencil assembly
# --------------------------------------------------------------------------

def _grid_coords(N: int):
    i = np.arange(N**3, dtype=np.int64)
    return i % N, (i // N) % N, i // (N * N)


def _stencil_csr(N: int, offsets, offdiag_w, diag) -> CSR:
    """Assemble a stencil operator on an N^3 grid.

    ``offsets``: list of (dx,dy,dz) sorted by linear offset dx+N*dy+N*N*dz,
    including (0,0,0).  ``offdiag_w[k]`` is an [n] array (or scalar) of the
    coupling *weight* for offset k (the matrix entry is ``-weight``);
    ``diag`` is the [n] diagonal.  Entries whose neighbour falls outside the
    grid are dropped.  Row-major flattening of the (n, len(offsets)) table keeps
    the columns of each row in ascending order.
    """
    n = N**3
    x, y, z = _grid_coords(N)
    k = len(offsets)
    valid = np.empty((n, k), dtype=bool)
    cols = np.empty((n, k), dtype=np.int32)
    vals = np.empty((n, k), dtype=np.float64)
    idx = np.arange(n, dtype=np.int64)
    for t, (dx, dy, dz) in enumerate(offsets):
        v = (x + dx >= 0) & (x + dx < N) & (y + dy >= 0) & (y + dy < N) & (z + dz >= 0) & (z + dz < N)
        valid[:, t] = v
        cols[:, t] = (idx + dx + N * dy + N * N * dz).astype(np.int32)
        if (dx, dy, dz) == (0, 0, 0):
            vals[:, t] = diag
        else:
            vals[:, t] = -np.broadcast_to(offdiag_w[t], (n,))
    del x, y, z, idx
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(valid.sum(1), out=rp[1:])
    col = cols[valid]
    val = vals[valid]
    del cols, vals, valid
    return CSR(n, rp.astype(np.int32), col, val)


def _offsets7(N):
    offs = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    return sorted(offs, key=lambda d: d[0] + N * d[1] + N * N * d[2])


def _offsets27(N):
    offs = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    return sorted(offs, key=lambda d: d[0] + N * d[1] + N * N * d[2])


def poisson7(N: int) -> CSR:
    """3D 7-point constant-coefficient Poisson, Dirichlet: a_ii = 6, a_ij = -1 to each in-grid face neighbour."""
    offs = _offsets7(N)
    w = [1.0 if d != (0, 0, 0) else 0.0 for d in offs]
    A = _stencil_csr(N, offs, w, 6.0)
    A.meta = {"kind": "poisson7", "N": N}
    return A


def vardens7(N: int, seed_rho: int = 2, seed_cut: int = 3, cut_frac: float = 0.05, with_cuts: bool = True) -> CSR:
    """3D 7-point variable-density Poisson with cut cells (the PeleLM-like operator).

    Cell density rho = 10^U(-3,3) (seed ``seed_rho``).  A Bernoulli(``cut_frac``)
    mask marks cut cells, each with one fraction f = 10^U(-8,0) serving as its
    volume/area fraction (seed ``seed_cut``); other cells have f = 1.  The face
    between cells a and b gets weight alpha*beta with beta the harmonic mean
    2 rho_a rho_b / (rho_a + rho_b) and alpha = min(f_a, f_b); the entry is
    -alpha*beta.  A boundary face of cell c adds f_c*rho_c to the diagonal.  The
    diagonal is the sum of the cell's face weights.  The result is a symmetric,
    irreducibly diagonally dominant M-matrix whose coefficients span many
    orders of magnitude.
    """
    n = N**3
    rng = np.random.default_rng(seed_rho)
    rho = 10.0 ** rng.uniform(-3.0, 3.0, n)
    f = np.ones(n)
    if with_cuts:
        rng2 = np.random.default_rng(seed_cut)
        cut = rng2.random(n) < cut_frac
        f[cut] = 10.0 ** rng2.uniform(-8.0, 0.0, int(cut.sum()))
    x, y, z = _grid_coords(N)
    offs = _offsets7(N)
    idx = np.arange(n, dtype=np.int64)
    weights = []
    diag = np.zeros(n)
    for (dx, dy, dz) in offs:
        if (dx, dy, dz) == (0, 0, 0):
            weights.append(0.0)
            continue
        inside = (x + dx >= 0) & (x + dx < N) & (y + dy >= 0) & (y + dy < N) & (z + dz >= 0) & (z + dz < N)
        nb = np.where(inside, idx + dx + N * dy + N * N * dz, idx)
        rb = rho[nb]
        beta = 2.0 * rho * rb / (rho + rb)
        alpha = np.minimum(f, f[nb])
        w = np.where(inside, alpha * beta, 0.0)
        weights.append(w)
        diag += np.where(inside, w, f * rho)
    A = _stencil_csr(N, offs, weights, diag)
    A.meta = {"kind": "vardens7", "N": N, "seed_rho": seed_rho, "seed_cut": seed_cut, "with_cuts": with_cuts}
    return A


def aniso27(N: int, ratio: float = 1.0e3) -> CSR:
    """3D 27-point anisotropic operator, anisotropy ``ratio`` along z.

    For offset d in {-1,0,1}^3 \\ 0 the coupling weight is
    w(d) = (dx^2 + dy^2 + ratio*dz^2) / |d|^4; a_{i,i+d} = -w(d) in-grid and
    a_ii = sum over all 26 offsets of w(d) (Dirichlet).  Symmetric positive
    definite M-matrix; the z-face to x-face weight ratio is ``ratio``.
    """
    offs = _offsets27(N)
    w = []
    for (dx, dy, dz) in offs:
        r2 = dx * dx + dy * dy + dz * dz
        w.append(0.0 if r2 == 0 else (dx * dx + dy * dy + ratio * dz * dz) / float(r2 * r2))
    diag = float(sum(w))
    A = _stencil_csr(N, offs, w, diag)
    A.meta = {"kind": "aniso27", "N": N, "ratio": ratio}
    return A


def permuted_longrange7(N: int, seed: int = 1, frac: float = 0.1, wmax: float = 1.0e-2, coo: bool = False) -> CSR:
    """7-point 256^3-style operator with random long-range couplings, symmetrically permuted.

    Start from the constant-coefficient 7-point grid (diagonal 6, face weight 1).
    With ``rng = default_rng(seed)`` draw, in this order: the permutation
    pi = rng.permutation(n); floor(frac*|E|) distinct grid edges (a<b) chosen
    uniformly without replacement; for each chosen edge a partner c uniform in
    [0,n) with c != a, c not a grid neighbour of a and {a,c} not already a new
    pair (redrawn until valid); then weights w ~ U(0, wmax).  Each chosen edge
    (a,b) is replaced by the coupling (a,c) with entry -w on both sides.  The
    diagonal stays 6.  Finally the matrix is permuted symmetrically, row r of
    the result being row pi[r] of the unpermuted matrix (with columns mapped
    the same way).  ``coo=True`` assembles the same matrix through a plain
    COO sort (slow; used to check the fast construction).
    """
    n = N**3
    rng = np.random.default_rng(seed)
    pi = rng.permutation(n).astype(np.int64)
    x, y, z = _grid_coords(N)
    idx = np.arange(n, dtype=np.int64)
    # grid edges (a, b), a < b: x-, y- and z-edges in that order
    ex = idx[x < N - 1]
    ey = idx[y < N - 1]
    ez = idx[z < N - 1]
    ea = np.concatenate([ex, ey, ez])
    eb = np.concatenate([ex + 1, ey + N, ez + N * N])
    del ex, ey, ez
    E = ea.shape[0]
    k = int(np.floor(frac * E))
    chosen = rng.choice(E, size=k, replace=False)
    ca, cb = ea[chosen], eb[chosen]
    keep = np.ones(E, dtype=bool)
    keep[chosen] = False
    ga, gb = ea[keep], eb[keep]
    chosen_idx = chosen
    del ea, eb, keep

    def is_grid_nb(a, c):
        d = np.abs(a - c)
        ax, ay, az = a % N, (a // N) % N, a // (N * N)
        cx, cy, cz = c % N, (c // N) % N, c // (N * N)
        man = np.abs(ax - cx) + np.abs(ay - cy) + np.abs(az - cz)
        return (man == 1) & ((d == 1) | (d == N) | (d == N * N))

    c = rng.integers(0, n, size=k, dtype=np.int64)
    todo = np.arange(k)
    for _ in range(64):
        bad = (c[todo] == ca[todo]) | is_grid_nb(ca[todo], c[todo])
        # duplicate unordered pairs among the new couplings
        lo = np.minimum(ca, c)
        hi = np.maximum(ca, c)
        key = lo * n + hi
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup_sorted = np.zeros(k, dtype=bool)
        dup_sorted[1:] = ks[1:] == ks[:-1]
        dup = np.zeros(k, dtype=bool)
        dup[order] = dup_sorted
        bad = bad | dup[todo]
        todo = todo[bad]
        if todo.size == 0:
            break
        c[todo] = rng.integers(0, n, size=todo.size, dtype=np.int64)
    else:  # pragma: no cover - astronomically unlikely
        raise RuntimeError("could not draw valid long-range partners")
    w = rng.uniform(0.0, wmax, size=k)
    if coo:
        # COO of the unpermuted symmetric matrix (plain reference construction)
        rows = np.concatenate([idx, ga, gb, ca, c])
        cols = np.concatenate([idx, gb, ga, c, ca])
        vals = np.concatenate([np.full(n, 6.0), -np.ones(ga.size), -np.ones(gb.size), -w, -w])
        inv = np.empty(n, dtype=np.int64)
        inv[pi] = np.arange(n, dtype=np.int64)
        A = _coo_to_csr(n, inv[rows], inv[cols], vals)
        A.meta = {"kind": "permuted_longrange7", "N": N, "seed": seed, "frac": frac}
        return A
    del ga, gb
    # Fast construction: a padded table of each unpermuted row (grid slots
    # -z,-y,-x,diag,+x,+y,+z, then long-range partners), columns mapped through
    # the inverse permutation, rows permuted, each short row sorted.
    nxe = N * N * (N - 1)  # edges per direction
    present = np.ones((3, n), dtype=bool)  # present[d][a]: edge (a, a+step_d) kept
    present[0, x == N - 1] = False
    present[1, y == N - 1] = False
    present[2, z == N - 1] = False
    # chosen edge indices were drawn over [x-edges | y-edges | z-edges]
    d_of = (chosen_idx // nxe).astype(np.int64)
    present[d_of, ca] = False
    steps = (1, N, N * N)
    nodes = np.concatenate([ca, c])
    deg = np.bincount(nodes, minlength=n)
    maxdeg = int(deg.max()) if deg.size else 0
    K = 7 + maxdeg
    tcol = np.full((n, K), -1, dtype=np.int64)
    tval = np.zeros((n, K))
    for slot, (dd, sign) in enumerate([(2, -1), (1, -1), (0, -1)]):
        st = steps[dd]
        ok = np.zeros(n, dtype=bool)
        ok[st:] = present[dd, :-st] if st < n else False
        tcol[:, slot] = np.where(ok, idx - st, -1)
        tval[:, slot] = np.where(ok, -1.0, 0.0)
    tcol[:, 3] = idx
    tval[:, 3] = 6.0
    for slot, dd in zip((4, 5, 6), (0, 1, 2)):
        st = steps[dd]
        ok = present[dd]
        tcol[:, slot] = np.where(ok, idx + st, -1)
        tval[:, slot] = np.where(ok, -1.0, 0.0)
    del present, x, y, z
    partners = np.concatenate([c, ca])
    ww = np.concatenate([w, w])
    order = np.argsort(nodes, kind="stable")
    nodes_s = nodes[order]
    first = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=first[1:])
    rank = np.arange(nodes_s.size) - first[nodes_s]
    tcol[nodes_s, 7 + rank] = partners[order]
    tval[nodes_s, 7 + rank] = -ww[order]
    del nodes, partners, ww, order, nodes_s, rank
    inv = np.empty(n, dtype=np.int64)
    inv[pi] = np.arange(n, dtype=np.int64)
    tcol = tcol[pi]
    tval = tval[pi]
    newc = np.where(tcol >= 0, inv[np.maximum(tcol, 0)], n)
    del tcol
    srt = np.argsort(newc, axis=1, kind="stable")
    newc = np.take_along_axis(newc, srt, axis=1)
    tval = np.take_along_axis(tval, srt, axis=1)
    del srt
    valid = newc < n
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(valid.sum(1), out=rp[1:])
    A = CSR(n, rp.astype(np.int32), newc[valid].astype(np.int32), tval[valid])
    A.meta = {"kind": "permuted_longrange7", "N": N, "seed": seed, "frac": frac}
    return A


def _coo_to_csr(n, rows, cols, vals) -> CSR:
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=n)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    return CSR(n, rp.astype(np.int32), cols.astype(np.int32), vals.astype(np.float64))


# --------------------------------------------------------------------------
# small random matrices for pins and edge cases
# --------------------------------------------------------------------------

def random_mmatrix(n: int, density: float, seed: int, sym: bool = False, dominance: float = 1.1) -> CSR:
    """Random sparse M-matrix: off-diagonals -U(0,1) on a random pattern, diagonal
    = ``dominance`` x (larger of row and column off-diagonal sums) + 0.1, so it is
    strictly diagonally dominant by rows and by columns."""
    rng = np.random.default_rng(seed)
    M = np.where(rng.random((n, n)) < density, -rng.random((n, n)), 0.0)
    np.fill_diagonal(M, 0.0)
    if sym:
        M = np.minimum(M, M.T)
    rs = -M.sum(1)
    cs = -M.sum(0)
    np.fill_diagonal(M, dominance * np.maximum(rs, cs) + 0.1)
    return CSR.from_dense(M)


def tridiag(n: int, a: float = -1.0, d: float = 2.0) -> CSR:
    """Tridiagonal (a, d, a) matrix."""
    M = np.diag(np.full(n, d)) + np.diag(np.full(n - 1, a), 1) + np.diag(np.full(n - 1, a), -1)
    return CSR.from_dense(M)


# --------------------------------------------------------------------------
# vectors
# --------------------------------------------------------------------------

def rhs(n: int, seed: int = 0) -> np.ndarray:
    """b ~ U(-1, 1) with ``default_rng(seed)``."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    A: CSR
    b: np.ndarray
    factor: str  # "ilu0" | "iluk" | "ilut"
    factor_params: dict
    outer: int
    m_L: int
    m_U: int
    mixed: bool = False


def workload(name: str, N: int | None = None) -> Workload:
    """Build one of the named synthetic workloads (optionally at a reduced grid side N).

    * ``poisson32``    7-pt Poisson, ILU(0), 1 outer x 3 inner (N=32, n=32768)
    * ``vardens128``   7-pt variable density with cut cells, ILU(1), 1 x 3 (N=128, n=2.1M)
    * ``aniso200``     27-pt anisotropic 1e3 along z, ILUT(1e-3, 20), 2 x 4 (N=200, n=8M)
    * ``perm256``      7-pt permuted with long-range couplings, ILU(0), FP32 factors, 1 x 3 (N=256, n=16.8M)
    """
    if name == "poisson32":
        N = N or 32
        A = poisson7(N)
        return Workload(name, A, rhs(A.n, 0), "ilu0", {}, 1, 3, 3)
    if name == "vardens128":
        N = N or 128
        A = vardens7(N)
        return Workload(name, A, rhs(A.n, 0), "iluk", {"k": 1}, 1, 3, 3)
    if name == "aniso200":
        N = N or 200
        A = aniso27(N)
        return Workload(name, A, rhs(A.n, 0), "ilut", {"tau": 1e-3, "p": 20}, 2, 4, 4)
    if name == "perm256":
        N = N or 256
        A = permuted_longrange7(N, seed=1)
        return Workload(name, A, rhs(A.n, 0), "ilu0", {}, 1, 3, 3, mixed=True)
    raise KeyError(name)
