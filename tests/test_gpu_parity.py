"""GPU parity: the HIP path through the C-ABI against the FP64 oracle, on
seeded inputs that span several workgroups and end in a ragged tail.

Tolerances: FP64 path 1e-12 relative, mixed path 1e-5 relative to the FP64
oracle (both element by element against the output's max norm, and norm-wise).
Where the kernel sums each row in the oracle's order (CSR-stream sweeps, the
row scaling) the result is also checked to be bit-identical."""
import numpy as np
import pytest

from paper_2111_09512_amd import workloads as W
from tests.gpu_common import F64_TOL, MIXED_TOL, Case, assert_close, dev, host, need_gpu, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    need_gpu()
    from paper_2111_09512_amd import binding

    return binding


@pytest.fixture(scope="module")
def ctx(B):
    return B.Context()


# None: sliced copies (the default: diagonal slices where every row lies on a few
# diagonals, else row patterns); "rowpat": row patterns even there
KERNELS = [None, "rowpat", "sliced8", "sliced_loop", "sliced16", "sliced32", "stream", "win", "stream16", "stream32",
           "blocked", "vector"]

SMALL = {
    "poisson17": (lambda: W.poisson7(17), "ilu0", {}),
    "vardens13_ilu1": (lambda: W.vardens7(13), "iluk", {"k": 1}),
    "aniso11_ilut": (lambda: W.aniso27(11), "ilut", {"tau": 1e-3, "p": 20}),
    "perm9": (lambda: W.permuted_longrange7(9, seed=1), "ilu0", {}),
}


@pytest.fixture(scope="module")
def cases(orc, B, ctx):
    out = {}
    for name, (make, kind, params) in SMALL.items():
        out[name] = Case(orc, B, ctx, make(), kind, params, fp32=True)
    return out


# --------------------------------------------------------------------------
# row scaling (eqs. extractD, newD)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", list(SMALL))
def test_scale_factors_bitwise(cases, name):
    say("scale", name)
    c = cases[name]
    F = c.F
    np.testing.assert_array_equal(host(F.Us.row_ptr), c.Us.row_ptr)
    np.testing.assert_array_equal(host(F.Us.col_idx), c.Us.col)
    np.testing.assert_array_equal(host(F.Us.val), c.Us.val)
    np.testing.assert_array_equal(host(F.d), c.d)
    np.testing.assert_array_equal(host(F.dinv), c.dinv)
    np.testing.assert_array_equal(host(F.Ls_val32), c.Ls.val.astype(np.float32))
    np.testing.assert_array_equal(host(F.Us_val32), c.Us.val.astype(np.float32))


def test_scale_factors_errors(B, ctx):
    say("scale errors")
    U = W.CSR.from_dense(np.array([[2.0, 1.0, 0.0], [0.0, 1.0, 3.0], [0.0, 0.0, 1.0]]))
    U.val[U.row_ptr[1]] = 0.0
    L = W.CSR.from_dense(np.zeros((3, 3)))
    L.row_ptr[:] = 0
    with pytest.raises(B.SiluError) as e:
        ctx.ilu_scale_factors(B.Csr.from_host(L), B.Csr.from_host(U))
    assert e.value.status == -4 and e.value.row == 1
    U2 = W.CSR.from_dense(np.array([[2.0, 1.0, 0.0], [0.0, 0.0, 3.0], [0.0, 0.0, 1.0]]))  # row 1 lacks its diagonal
    with pytest.raises(B.SiluError) as e:
        ctx.ilu_scale_factors(B.Csr.from_host(L), B.Csr.from_host(U2))
    assert e.value.status == -3 and e.value.row == 1


# --------------------------------------------------------------------------
# the smoother, FP64
# --------------------------------------------------------------------------

SCHED = [(1, 3, 3), (2, 4, 4), (1, 1, 1), (1, 1, 3), (1, 3, 1), (3, 2, 5)]


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("sched", SCHED, ids=lambda s: "o%dL%dU%d" % s)
@pytest.mark.parametrize("name", list(SMALL))
def test_smooth_f64(orc, ctx, cases, name, sched, kernel):
    outer, mL, mU = sched
    say("smooth f64", name, sched, kernel)
    c = cases[name]
    b = W.rhs(c.A.n, 0)
    x0 = W.rhs(c.A.n, 7) if outer > 1 else np.zeros(c.A.n)
    ref = orc.smooth(c.A, c.Ls, c.Us, c.dinv, b, x0, outer, mL, mU)
    x = dev(x0)
    ctx.ilu_smooth(c.Ad, c.F, dev(b), x, outer, mL, mU, kernel=kernel)
    got = host(x)
    assert_close(got, ref, F64_TOL, f"{name} {sched} {kernel}")
    if kernel != "vector":  # same per-row summation order as the oracle
        np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("name", list(SMALL))
def test_smooth_direct(orc, ctx, cases, name):
    say("smooth direct", name)
    c = cases[name]
    b = W.rhs(c.A.n, 0)
    x0 = W.rhs(c.A.n, 3)
    ref = orc.smooth(c.A, c.Ls, c.Us, c.dinv, b, x0, 2, 0, 0, direct=True)
    x = dev(x0)
    ctx.ilu_smooth(c.Ad, c.F, dev(b), x, 2, 1, 1, direct=True)
    got = host(x)
    assert_close(got, ref, F64_TOL, f"direct {name}")


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("sched", [(1, 3, 3), (2, 4, 4), (1, 1, 1), (1, 2, 1), (1, 1, 2)], ids=lambda s: "o%dL%dU%d" % s)
@pytest.mark.parametrize("name", list(SMALL))
def test_smooth_mixed(orc, ctx, cases, name, sched, kernel):
    """FP32-inner form: within 1e-5 of the FP64 oracle, and equal to the
    oracle's emulation of the same rounding points up to FP32 summation order."""
    outer, mL, mU = sched
    say("smooth mixed", name, sched, kernel)
    c = cases[name]
    b = W.rhs(c.A.n, 0)
    x0 = np.zeros(c.A.n)
    ref64 = orc.smooth(c.A, c.Ls, c.Us, c.dinv, b, x0, outer, mL, mU)
    ref32 = orc.smooth_mixed(c.A, c.Ls, c.Us, c.dinv, b, x0, outer, mL, mU)
    x = dev(x0)
    ctx.ilu_smooth(c.Ad, c.F, dev(b), x, outer, mL, mU, mixed=True, kernel=kernel)
    got = host(x)
    err = rel_err(got, ref64)
    say("  mixed rel err vs fp64 oracle", f"{err:.3e}")
    assert_close(got, ref64, MIXED_TOL, f"mixed {name} {sched}")
    if kernel != "vector":
        np.testing.assert_array_equal(got, ref32)
    else:
        assert rel_err(got, ref32) <= 1e-6


@pytest.mark.parametrize("sched", [(1, 3, 3), (1, 1, 1), (1, 3, 1), (2, 2, 4)], ids=lambda s: "o%dL%dU%d" % s)
def test_smooth_unscaled(orc, B, ctx, sched):
    """The unscaled variant z <- y - (U - I) z (Section 6.1): same arithmetic
    as the oracle, compared relative to the magnitude the iteration reaches."""
    outer, mL, mU = sched
    say("unscaled", sched)
    A = W.vardens7(9)
    c = Case(orc, B, ctx, A, "iluk", {"k": 1}, scale=False)
    np.testing.assert_array_equal(host(c.F.Us.val), c.U.val[np.repeat(np.arange(A.n), np.diff(c.U.row_ptr)) != c.U.col])
    b = W.rhs(A.n, 0)
    ref = orc.smooth_unscaled(A, c.Ls, c.U, b, np.zeros(A.n), outer, mL, mU)
    x = dev(np.zeros(A.n))
    ctx.ilu_smooth(c.Ad, c.F, dev(b), x, outer, mL, mU)
    got = host(x)
    np.testing.assert_array_equal(got, ref)


# --------------------------------------------------------------------------
# triangular solves and level analysis (Section 4)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", list(SMALL))
def test_trisolve_direct(orc, B, ctx, cases, name):
    """Level-scheduled substitution (several lanes per row for longer rows)
    against the oracle's sequential substitution."""
    say("trisolve_direct", name)
    c = cases[name]
    rhs = W.rhs(c.A.n, 5)
    for T, Td, uplo, unit in ((c.Ls, c.Ld, B.SILU_LOWER, True), (c.Us, c.F.Us, B.SILU_UPPER, True),
                              (c.U, c.Ud, B.SILU_UPPER, False)):
        ref = orc.trisolve(T, "L" if uplo == B.SILU_LOWER else "U", unit, rhs)
        got = host(ctx.trisolve_direct(Td, uplo, B.SILU_UNIT if unit else B.SILU_NONUNIT, dev(rhs)))
        assert_close(got, ref, F64_TOL, f"direct {name} {uplo} unit={unit}")


@pytest.mark.parametrize("name", list(SMALL))
def test_analyze_levels(orc, B, ctx, cases, name):
    say("analyze", name)
    c = cases[name]
    for T, Td, uplo in ((c.Ls, c.Ld, "L"), (c.Us, c.F.Us, "U")):
        lev, depth = orc.levels(T, uplo)
        d, rows = ctx.silu_analyze(Td, B.SILU_LOWER if uplo == "L" else B.SILU_UPPER)
        assert d == depth
        np.testing.assert_array_equal(rows, np.bincount(lev, minlength=depth))


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("name", list(SMALL))
def test_trisolve_iter(orc, B, ctx, cases, name, kernel):
    """m Richardson steps against the oracle, and m = depth (nilpotence) against
    the level-scheduled direct solve."""
    say("trisolve_iter", name, kernel)
    c = cases[name]
    rhs = W.rhs(c.A.n, 6)
    for T, Td, uplo in ((c.Ls, c.Ld, "L"), (c.Us, c.F.Us, "U")):
        for m in (1, 2, 5):
            ref = orc.richardson(T, c.dinv * rhs if uplo == "U" else rhs, m)
            got = host(ctx.trisolve_iter(Td, dev(rhs), m, dinv=c.F.dinv if uplo == "U" else None, kernel=kernel))
            assert_close(got, ref, F64_TOL, f"iter {name} {uplo} m={m}")
        depth, _ = ctx.silu_analyze(Td, B.SILU_LOWER if uplo == "L" else B.SILU_UPPER)
        exact = orc.trisolve(T, uplo, True, rhs)
        got = host(ctx.trisolve_iter(Td, dev(rhs), depth, kernel=kernel))
        assert_close(got, exact, F64_TOL, f"nilpotence {name} {uplo}")
        if kernel != "vector":
            np.testing.assert_array_equal(got, exact)
        direct = host(ctx.trisolve_direct(Td, B.SILU_LOWER if uplo == "L" else B.SILU_UPPER, B.SILU_UNIT, dev(rhs)))
        assert_close(direct, got, F64_TOL, f"iterative vs direct {name} {uplo}")


# --------------------------------------------------------------------------
# edge cases
# --------------------------------------------------------------------------

def test_edge_single_row(orc, B, ctx):
    say("edge n=1")
    A = W.CSR.from_dense(np.array([[4.0]]))
    c = Case(orc, B, ctx, A, "ilu0", {}, fp32=True)
    b = np.array([2.0])
    for mixed in (False, True):
        x = dev(np.zeros(1))
        ctx.ilu_smooth(c.Ad, c.F, dev(b), x, 2, 3, 3, mixed=mixed)
        assert host(x)[0] == orc.smooth(A, c.Ls, c.Us, c.dinv, b, np.zeros(1), 2, 3, 3)[0] == 0.5


def test_edge_diagonal_matrix_empty_factors(orc, B, ctx):
    """A diagonal A has empty strict factors (nnz = 0): one step is exact."""
    say("edge diagonal")
    d = np.linspace(1.0, 3.0, 1000)
    A = W.CSR.from_dense(np.diag(d))
    c = Case(orc, B, ctx, A, "ilu0", {}, fp32=True)
    assert c.Ls.nnz == 0 and c.Us.nnz == 0
    b = W.rhs(A.n, 0)
    x = dev(np.zeros(A.n))
    ctx.ilu_smooth(c.Ad, c.F, dev(b), x, 1, 3, 3)
    np.testing.assert_array_equal(host(x), orc.smooth(A, c.Ls, c.Us, c.dinv, b, np.zeros(A.n), 1, 3, 3))
    x = dev(np.zeros(A.n))
    ctx.ilu_smooth(c.Ad, c.F, dev(b), x, 1, 1, 1, direct=True)
    np.testing.assert_allclose(host(x), b / d, rtol=1e-15)


@pytest.mark.parametrize("kernel", KERNELS)
def test_edge_long_rows(orc, B, ctx, kernel):
    """Rows far longer than one LDS chunk of the CSR-stream kernel (several
    chunks per workgroup) next to empty rows."""
    say("edge long rows", kernel)
    n = 3000
    rng = np.random.default_rng(1)
    M = np.diag(np.full(n, 4.0 * n))
    M[n - 1, : n - 1] = -rng.random(n - 1)  # one full lower row
    M[0, 1:] = -rng.random(n - 1)           # one full upper row
    M[n // 2, : n // 2] = -rng.random(n // 2)
    A = W.CSR.from_dense(M)
    c = Case(orc, B, ctx, A, "ilu0", {}, fp32=True)
    b = W.rhs(n, 0)
    ref = orc.smooth(A, c.Ls, c.Us, c.dinv, b, np.zeros(n), 1, 3, 3)
    x = dev(np.zeros(n))
    ctx.ilu_smooth(c.Ad, c.F, dev(b), x, 1, 3, 3, kernel=kernel)
    assert_close(host(x), ref, F64_TOL, "long rows")
    if kernel != "vector":
        np.testing.assert_array_equal(host(x), ref)


def test_error_paths(B, ctx, cases):
    say("error paths")
    c = cases["poisson17"]
    n = c.A.n
    b, x = dev(W.rhs(n, 0)), dev(np.zeros(n))
    with pytest.raises(B.SiluError) as e:
        ctx.ilu_smooth(c.Ad, c.F, b, x, 0, 3)
    assert e.value.status == -1
    with pytest.raises(B.SiluError) as e:
        ctx.ilu_smooth(c.Ad, c.F, b, x, 1, 0)
    assert e.value.status == -1
    small = __import__("torch").empty(1024, dtype=__import__("torch").uint8, device="cuda")
    with pytest.raises(B.SiluError) as e:
        ctx.ilu_smooth(c.Ad, c.F, b, x, 1, 3, ws=small)
    assert e.value.status == -6
    F32less = B.Factors(c.F.Ls, c.F.Us, c.F.d, c.F.dinv, None, None, True)
    with pytest.raises(B.SiluError) as e:
        ctx.ilu_smooth(c.Ad, F32less, b, x, 1, 3, mixed=True)
    assert e.value.status == -8
    bad = b.clone()
    bad[n // 3] = float("nan")
    with pytest.raises(B.SiluError) as e:
        ctx.ilu_smooth(c.Ad, c.F, bad, x, 1, 3, check_finite=True)
    assert e.value.status == -5
    # VALIDATE catches an unsorted row
    Abad = B.Csr(c.Ad.row_ptr.clone(), c.Ad.col_idx.clone(), c.Ad.val.clone())
    cols = Abad.col_idx.cpu()
    cols[1], cols[2] = cols[2].item(), cols[1].item()
    Abad.col_idx.copy_(cols.cuda())
    with pytest.raises(B.SiluError) as e:
        ctx.ilu_smooth(Abad, c.F, b, x, 1, 3, validate=True)
    assert e.value.status == -3


def test_timing_stats(B, ctx, cases):
    say("timing stats")
    c = cases["aniso11_ilut"]
    n = c.A.n
    ctx.stats_reset()
    ctx.set_timing(True)
    x = dev(np.zeros(n))
    ctx.ilu_smooth(c.Ad, c.F, dev(W.rhs(n, 0)), x, 2, 4, 4)
    ctx.set_timing(False)
    st = ctx.stats()
    total = sum(v["launches"] for v in st.values())
    assert total == 2 * (1 + 3 + 3)
    assert all(v["ms"] > 0 and v["bytes"] > 0 for v in st.values() if v["launches"])
    ctx.stats_reset()


@pytest.mark.parametrize("kernel", KERNELS)
def test_many_row_blocks_per_workgroup(orc, B, ctx, kernel):
    """More row blocks than resident workgroups, so each workgroup of the
    pipelined kernel walks a slab of blocks, with rows longer than one LDS
    chunk scattered among short ones (strictly lower T, n = 400000)."""
    say("many row blocks", kernel)
    n = 400_000
    rng = np.random.default_rng(11)
    i = np.arange(n)
    step = 1 + i % 7  # row i reads columns i-1-k*step, k < len_i
    lens = rng.integers(0, 12, n)
    for r in (5000, 123457, 300001, n - 1):  # rows longer than one LDS chunk
        lens[r] = 2500 + r % 700
        step[r] = 1
    lens = np.where(i == 0, 0, np.minimum(lens, (i - 1) // step + 1))
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    row = np.repeat(i, lens)
    k = np.arange(rp[-1]) - rp[row]
    col = (row - 1 - (lens[row] - 1 - k) * step[row]).astype(np.int32)
    assert col.min() >= 0 and np.all(col < row)
    T = W.CSR(n, rp.astype(np.int32), col, -rng.random(rp[-1]) / 20.0)
    Td = B.Csr.from_host(T)
    rhs = W.rhs(n, 3)
    for m in (1, 3):
        ref = orc.richardson(T, rhs, m)
        got = host(ctx.trisolve_iter(Td, dev(rhs), m, kernel=kernel))
        assert_close(got, ref, F64_TOL, f"many blocks m={m}")
        if kernel != "vector":
            np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("name", ["vardens13_ilu1", "aniso11_ilut"])
def test_level_graph_replays(orc, B, ctx, cases, name):
    """The level sequence is captured once into a hipGraph and replayed: every
    replay, with eager work and synchronizations in between, matches the
    oracle's substitution and equals the plain-launch path bit for bit."""
    import torch

    say("graph replays", name)
    c = cases[name]
    n = c.A.n
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    for rep in range(4):
        rhs = W.rhs(n, 20 + rep)
        ref = orc.trisolve(c.Us, "U", True, rhs)
        rd = dev(rhs)
        ctx.trisolve_direct(c.F.Us, B.SILU_UPPER, B.SILU_UNIT, rd, out=out)
        got = host(out)
        assert_close(got, ref, F64_TOL, f"graph replay {rep}")
        junk = torch.randn(4096, device="cuda").cumsum(0)  # eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(junk).all()
        plain = ctx.trisolve_direct(c.F.Us, B.SILU_UPPER, B.SILU_UNIT, rd, graph=False)
        np.testing.assert_array_equal(host(plain), got)
    b = W.rhs(n, 0)
    x0 = W.rhs(n, 3)
    ref = orc.smooth(c.A, c.Ls, c.Us, c.dinv, b, x0, 1, 0, 0, direct=True)
    bd = dev(b)
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    first = None
    for rep in range(3):
        x.copy_(dev(x0))
        ctx.ilu_smooth(c.Ad, c.F, bd, x, 1, 1, 1, direct=True)
        got = host(x)
        assert_close(got, ref, F64_TOL, f"direct smoother replay {rep}")
        if first is None:
            first = got
        np.testing.assert_array_equal(got, first)
        torch.cuda.synchronize()


def test_cached_analyses_follow_matrix_lifetime(orc, B, ctx):
    """Analyses are cached by pointer; freeing a matrix releases them, so a new
    matrix of the same size at the same addresses gets fresh ones."""
    import gc

    import torch

    say("cache lifetime")
    n = 3000
    rhs = W.rhs(n, 1)
    for seed in range(3):
        rng = np.random.default_rng(seed)
        M = np.tril(np.where(rng.random((n, n)) < 0.002, -rng.random((n, n)), 0.0), -1)
        # same nnz every time: keep exactly 4000 strictly-lower entries
        rows, cols = np.nonzero(M)
        keep = rng.choice(rows.size, 4000, replace=False)
        D = np.zeros((n, n))
        D[rows[keep], cols[keep]] = -rng.random(4000) / 10.0
        T = W.CSR.from_dense(D)
        Td = B.Csr.from_host(T)
        for m in (2, 5):
            np.testing.assert_array_equal(host(ctx.trisolve_iter(Td, dev(rhs), m)), orc.richardson(T, rhs, m))
        assert_close(host(ctx.trisolve_direct(Td, B.SILU_LOWER, B.SILU_UNIT, dev(rhs))),
                     orc.trisolve(T, "L", True, rhs), F64_TOL, "direct after reuse of addresses")
        del Td
        gc.collect()
        torch.cuda.synchronize()


@pytest.mark.parametrize("name", ["poisson17", "aniso11_ilut", "perm9"])
def test_outer_convergence_counts(orc, B, ctx, cases, name):
    """Repeated smoothing on the GPU reaches ||b - A x|| / ||b|| < 1e-8 (eq.
    relres) in the same number of outer steps as the oracle, for the FP64 and
    the FP32-inner forms, and the two forms need the same number of steps."""
    say("outer convergence", name)
    c = cases[name]
    b = W.rhs(c.A.n, 0)
    nb = np.linalg.norm(b)
    counts = {}
    for mixed in (False, True):
        k_ref, _, hist = orc.smooth_until(c.A, c.Ls, c.Us, c.dinv, b, np.zeros(c.A.n), 3, 3, 1e-8, 300, mixed=mixed)
        assert k_ref <= 300
        bd, x = dev(b), dev(np.zeros(c.A.n))
        k = 0
        while True:
            ctx.ilu_smooth(c.Ad, c.F, bd, x, 1, 3, 3, mixed=mixed)
            k += 1
            rel = np.linalg.norm(orc.residual(c.A, b, host(x))) / nb
            if rel < 1e-8 or k > 300:
                break
        assert k == k_ref, f"mixed={mixed}: GPU {k} steps, oracle {k_ref}"
        counts[mixed] = k
    assert counts[True] == counts[False]


def test_values_changed_in_place(orc, B, ctx):
    """The sliced copies hold values: changing A's or L's values in place is
    seen by the next call (the binding releases the stale copies)."""
    say("values changed in place")
    A = W.vardens7(11, seed_rho=3)
    Ls, U = orc.ilu0(A)
    d, dinv, Us = orc.scale_rows(U)
    Ad, Ld, Ud = B.Csr.from_host(A), B.Csr.from_host(Ls), B.Csr.from_host(U)
    F = ctx.ilu_scale_factors(Ld, Ud)
    b = W.rhs(A.n, 0)
    x = dev(np.zeros(A.n))
    ctx.ilu_smooth(Ad, F, dev(b), x, 1, 3, 3)
    np.testing.assert_array_equal(host(x), orc.smooth(A, Ls, Us, dinv, b, np.zeros(A.n), 1, 3, 3))
    Ad.val.mul_(2.0)  # in place on the device
    Ld.val.mul_(0.5)
    A2 = W.CSR(A.n, A.row_ptr, A.col, A.val * 2.0)
    L2 = W.CSR(Ls.n, Ls.row_ptr, Ls.col, Ls.val * 0.5)
    x = dev(np.zeros(A.n))
    ctx.ilu_smooth(Ad, F, dev(b), x, 1, 3, 3)
    np.testing.assert_array_equal(host(x), orc.smooth(A2, L2, Us, dinv, b, np.zeros(A.n), 1, 3, 3))


@pytest.mark.parametrize("kernel", [None, "sliced16", "sliced32", "stream", "stream32", "blocked", "win"])
@pytest.mark.parametrize("n", [2, 63, 64, 65, 127, 129, 255, 257, 1000])
def test_ragged_sizes_variable_rows(orc, B, ctx, n, kernel):
    """Row counts around the 64-row slice and the 256-row block, with row
    lengths from 0 to dozens in each factor (masked and unmasked slices side by
    side): FP64 and the FP32-inner form bit for bit against the oracle and its
    emulation."""
    rng = np.random.default_rng(n)
    M = np.zeros((n, n))
    for i in range(n):
        k = int(rng.integers(0, min(n, 40)))
        cols = rng.choice(n, size=k, replace=False)
        M[i, cols] = -rng.random(k)
    np.fill_diagonal(M, 0.0)
    M = M + M.T
    np.fill_diagonal(M, np.abs(M).sum(axis=1) + 1.0)
    A = W.CSR.from_dense(M)
    c = Case(orc, B, ctx, A, "ilu0", {}, fp32=True)
    b, x0 = W.rhs(n, 1), W.rhs(n, 2)
    ref = orc.smooth(A, c.Ls, c.Us, c.dinv, b, x0, 2, 3, 4)
    ref32 = orc.smooth_mixed(A, c.Ls, c.Us, c.dinv, b, x0, 2, 3, 4)
    for mixed, want in ((False, ref), (True, ref32)):
        x = dev(x0)
        ctx.ilu_smooth(c.Ad, c.F, dev(b), x, 2, 3, 4, mixed=mixed, kernel=kernel)
        np.testing.assert_array_equal(host(x), want)


@pytest.mark.parametrize("name", ["aniso11_ilut", "perm9"])
def test_run_twice_deterministic(orc, B, ctx, cases, name):
    """Every entry point gives the same bits when called twice on the same
    inputs (no atomics or arrival-order reductions anywhere on the path): the
    smoother under every kernel variant (including vector-CSR, whose shuffle
    reductions differ from the oracle's order but not from run to run), FP64
    and FP32-inner, the direct form, the polynomial Gauss-Seidel smoother and
    FGMRES."""
    say("run twice", name)
    c = cases[name]
    b, x0 = dev(W.rhs(c.A.n, 7)), dev(W.rhs(c.A.n, 8))

    def twice(fn):
        outs = []
        for _ in range(2):
            x = x0.clone()
            fn(x)
            outs.append(host(x))
        np.testing.assert_array_equal(outs[0], outs[1])

    for kernel in KERNELS:
        for mixed in (False, True):
            twice(lambda x: ctx.ilu_smooth(c.Ad, c.F, b, x, 2, 3, 4, mixed=mixed, kernel=kernel))
    twice(lambda x: ctx.ilu_smooth(c.Ad, c.F, b, x, 2, 1, 1, direct=True))
    G = ctx.gs_split(c.Ad, fp32=True)
    for mixed in (False, True):
        twice(lambda x: ctx.gs_smooth(c.Ad, G, b, x, 2, 3, mixed=mixed))
    twice(lambda x: ctx.fgmres(c.Ad, c.F, b, x, restart=10, max_iters=40, tol=1e-10))


def test_calibration_streams(B, ctx):
    """The bandwidth calibration kernels move the bytes they claim: the copy
    reproduces its source, the read stream's check words are the XOR of the
    16-byte vectors each lane read (two tiles and a grid-stride remainder)."""
    import torch

    say("calibration streams")
    rng = np.random.default_rng(11)
    nbytes = 3 * 49152
    words = rng.integers(0, 2**32, nbytes // 4, dtype=np.uint64).astype(np.uint32)
    src = torch.from_numpy(words.view(np.int32).copy()).cuda()
    dst = torch.zeros_like(src)
    ctx.stream_copy(src, dst)
    np.testing.assert_array_equal(host(dst), words.view(np.int32))
    out = torch.zeros(nbytes // 24 // 8, dtype=torch.int64, device="cuda")
    ctx.stream_read(src, out)
    v = words.reshape(3, 12, 256, 4)  # tile, vector k, lane, 32-bit word
    acc = np.bitwise_xor.reduce(v, axis=1).astype(np.uint64)  # [tile, lane, 4]
    want = ((acc[..., 0] ^ acc[..., 2]) << np.uint64(32)) | (acc[..., 1] ^ acc[..., 3])
    np.testing.assert_array_equal(host(out).view(np.uint64), want.reshape(-1))
    with pytest.raises(B.SiluError):
        ctx.stream_read(src[:1000], out)


def _patterned_lower(n, npat, rowlen, seed):
    """Strictly lower matrix whose rows follow `npat` offset patterns (each
    `rowlen` distinct offsets in [1, 4 rowlen]), assigned to rows at random; a
    row whose offsets would leave the matrix keeps only the ones that fit (a
    boundary pattern of its own)."""
    rng = np.random.default_rng(seed)
    pats = [np.sort(rng.choice(np.arange(1, 4 * rowlen + 1), size=rowlen, replace=False))[::-1] for _ in range(npat)]
    which = rng.integers(0, npat, size=n)
    rows, cols = [], []
    for i in range(n):
        c = i - pats[which[i]]
        c = c[c >= 0]
        rows.append(np.full(c.size, i))
        cols.append(c)
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    D = np.zeros((n, n))
    D[rows, cols] = -rng.random(rows.size) / (2.0 * rowlen)
    return W.CSR.from_dense(D)


@pytest.mark.parametrize("npat,rowlen", [(1, 5), (120, 8), (240, 12), (300, 6), (60, 32), (40, 33)])
def test_row_pattern_tables(orc, B, ctx, npat, rowlen):
    """Row-pattern sliced copies at their limits: one pattern, up to 256 (counting
    the boundary rows' own), more than 256 (the 1-byte diagonal codes instead),
    32 slots per row (eight groups, the most the pattern sweep takes) and 33 (the
    coded layout instead); every layout choice gives the oracle's Richardson
    iterates bit for bit."""
    say("row patterns", npat, rowlen)
    n = 1500
    T = _patterned_lower(n, npat, rowlen, seed=npat * 100 + rowlen)
    Td = B.Csr.from_host(T)
    rhs = W.rhs(n, 9)
    for m in (1, 3, 6):
        for kernel in (None, "sliced8"):
            np.testing.assert_array_equal(host(ctx.trisolve_iter(Td, dev(rhs), m, kernel=kernel)),
                                          orc.richardson(T, rhs, m))


def _banded(n, diags, seed, drop=0.0):
    """n x n matrix on the given diagonals (entries outside the matrix
    dropped), each entry kept with probability 1 - drop, values of both signs."""
    rng = np.random.default_rng(seed)
    D = np.zeros((n, n))
    for d in diags:
        i = np.arange(max(0, -d), min(n, n - d))
        keep = rng.random(i.size) >= drop
        D[i[keep], i[keep] + d] = rng.uniform(-1.0, 1.0, int(keep.sum())) / len(diags)
    return W.CSR.from_dense(D)


@pytest.mark.parametrize("n", [2, 3, 127, 128, 129, 255, 300, 1000])
@pytest.mark.parametrize("diags,drop", [((-130, -7, -1, 1, 2, 64, 129), 0.0), ((-3, -2, -1), 0.02),
                                        (tuple(range(-30, 0)), 0.0), ((-1, 1), 0.5)])
def test_diagonal_slices(orc, B, ctx, n, diags, drop):
    """Matrices on a few diagonals take the diagonal-slice copy (two rows per
    lane, 16-byte value and iterate loads, columns clamped at both ends of the
    matrix, rows past n in the last 128-row slice): the product and Richardson
    iterates equal the oracle's bit for bit, and those of the row-pattern copy
    (SILU_ROWPAT) and of the CSR stream; with 30 diagonals (above the 24 whose
    epilogue operands are loaded early), and with entries missing from a
    diagonal (zeros in its slots; too many and the copy is not used)."""
    say("diagonal slices", n, len(diags), drop)
    L = _banded(n, diags, seed=n + len(diags))
    Ld = B.Csr.from_host(L)
    x = W.rhs(n, 3)
    want = orc.spmv(L, x)
    for kernel in (None, "rowpat", "stream"):
        np.testing.assert_array_equal(host(ctx.spmv(Ld, dev(x), kernel=kernel)), want)
    if all(d < 0 for d in diags):  # strictly lower: Richardson iterates on it
        for m in (1, 2, 5):
            ref = orc.richardson(L, x, m)
            for kernel in (None, "rowpat"):
                np.testing.assert_array_equal(host(ctx.trisolve_iter(Ld, dev(x), m, kernel=kernel)), ref)


def _runs(n, starts, width, seed, drop=0.0):
    """n x n matrix on runs of `width` consecutive diagonals beginning at each
    offset in `starts` (entries outside the matrix dropped)."""
    diags = sorted({s + j for s in starts for j in range(width)})
    return _banded(n, diags, seed, drop), diags


@pytest.mark.parametrize("n", [3001, 64 * 70 + 17])
@pytest.mark.parametrize("starts,width,drop", [
    ((-1,), 1, 0.0),                                      # one window
    (tuple(-200 * k - 1 for k in range(1, 13)), 2, 0.0),  # twelve (the most), odd first offsets
    (tuple(-200 * k for k in range(1, 14)), 1, 0.0),      # thirteen: no windows, the gather body
    ((-300,), 65, 0.0),                                   # offsets w .. w + 64 (w even): one window, read to its end
    ((-301,), 64, 0.0),                                   # from an odd offset, rounded down: still one
    ((-300,), 66, 0.0),                                   # one offset more: two windows
    ((-700, -3), 3, 0.03),                                # missing entries: several row patterns
    ((-150, 1, 140), 3, 0.0),                             # both sides of the diagonal
])
def test_pattern_windows(orc, B, ctx, n, starts, width, drop):
    """Row-pattern copies whose offsets fall in runs: the windowed sweep (each
    slice's iterate windows staged in LDS, one load per window, slots read at
    lane + index) covers the slices whose windows lie inside the matrix, the
    gather body the slices at either end, those with an empty row (row 0 of a
    strictly lower matrix) and the ragged last one; product and Richardson
    iterates equal the oracle's bit for bit, for 1 to 12 windows and for 13
    (none kept), with runs reaching the last entry of a window from even and
    odd starts."""
    say("pattern windows", n, len(starts), width, drop)
    L, diags = _runs(n, starts, width, seed=n + width, drop=drop)
    Ld = B.Csr.from_host(L)
    x = W.rhs(n, 5)
    want = orc.spmv(L, x)
    for kernel in (None, "rowpat"):
        np.testing.assert_array_equal(host(ctx.spmv(Ld, dev(x), kernel=kernel)), want)
    if all(d < 0 for d in diags):
        for m in (1, 3):
            ref = orc.richardson(L, x, m)
            np.testing.assert_array_equal(host(ctx.trisolve_iter(Ld, dev(x), m, kernel="rowpat")), ref)


@pytest.mark.parametrize("n", [4000, 64 * 90 + 33])
@pytest.mark.parametrize("rare_rows", [(1000, 1001, 1063), (2000,), ()])
def test_pattern_windows_rare_run(orc, B, ctx, n, rare_rows):
    """A run of offsets that few slices need gets no window: the two common
    diagonals -1 and -2 are staged as one window, while the rows holding an
    entry on diagonal -700 (rows in one or two slices, far fewer than 1/16
    of them) send their slices to the gather body; every result equals the
    oracle's bit for bit, with and without such rows."""
    say("pattern windows, rare run", n, rare_rows)
    L, _ = _runs(n, (-2,), 2, seed=n)
    D = L.to_dense()
    rng = np.random.default_rng(n)
    for r in rare_rows:
        D[r, r - 700] = rng.uniform(-1.0, 1.0)
    M = W.CSR.from_dense(D)
    Md = B.Csr.from_host(M)
    x = W.rhs(n, 7)
    np.testing.assert_array_equal(host(ctx.spmv(Md, dev(x), kernel="rowpat")), orc.spmv(M, x))
    for m in (1, 3):
        np.testing.assert_array_equal(host(ctx.trisolve_iter(Md, dev(x), m, kernel="rowpat")), orc.richardson(M, x, m))


@pytest.mark.parametrize("shift", [0, 1])
def test_pattern_windows_unaligned_iterate(orc, B, ctx, shift):
    """An iterate that is not 16-byte aligned (a view one element into a
    larger tensor) takes the gather body instead of the windows; both give the
    oracle's product bit for bit."""
    import torch
    n = 3001
    say("pattern windows, unaligned iterate", shift)
    L, _ = _runs(n, (-300, -2), 3, seed=11)
    Ld = B.Csr.from_host(L)
    x = W.rhs(n, 9)
    big = torch.zeros(n + 1, dtype=torch.float64, device="cuda")
    big[shift:shift + n] = dev(x)
    xv = big[shift:shift + n]
    assert (xv.data_ptr() % 16 != 0) == bool(shift)
    np.testing.assert_array_equal(host(ctx.spmv(Ld, xv, kernel="rowpat")), orc.spmv(L, x))
