"""GPU parity of the Krylov solver around the smoother (FGMRES with the ILU
smoother as right preconditioner; eq. relres stopping rule; NRBE of eq.
nbre), of the product with A and of the dot product, against the oracle.

Tolerance of the FGMRES comparison: the GPU reduces dot products in a fixed
blocked order, the oracle in index order; the two differ by rounding of at
most n * eps relative per dot product (about 1e-12 here), amplified through
Gram-Schmidt and the small least-squares problem by at most the condition of
the preconditioned operator (tens here).  So the step counts must agree, the
residual histories to 1e-6 relative and the solutions to 1e-7 of their max
norm -- wide margins over those bounds."""
import numpy as np
import pytest
import torch

from paper_2111_09512_amd import workloads as W
from tests.gpu_common import assert_close, dev, host, need_gpu, say

pytestmark = pytest.mark.gpu

SMALL = {
    "poisson17": (lambda: W.poisson7(17), "ilu0", {}),
    "vardens13_ilu1": (lambda: W.vardens7(13), "iluk", {"k": 1}),
    "aniso11_ilut": (lambda: W.aniso27(11), "ilut", {"tau": 1e-3, "p": 20}),
    "perm9": (lambda: W.permuted_longrange7(9, seed=1), "ilu0", {}),
}


@pytest.fixture(scope="module")
def B():
    need_gpu()
    from paper_2111_09512_amd import binding

    return binding


@pytest.fixture(scope="module")
def ctx(B):
    return B.Context()


class KCase:
    def __init__(self, orc, B, ctx, A, kind, params):
        self.A = A
        self.Ls, U = orc.factor(A, kind, params)
        self.d, self.dinv, self.Us = orc.scale_rows(U)
        self.Ad, Ld, Ud = B.Csr.from_host(A), B.Csr.from_host(self.Ls), B.Csr.from_host(U)
        self.F = ctx.ilu_scale_factors(Ld, Ud, fp32=True)
        self.Ld, self.Ud = Ld, Ud
        torch.cuda.synchronize()


@pytest.fixture(scope="module")
def cases(orc, B, ctx):
    return {name: KCase(orc, B, ctx, make(), kind, params) for name, (make, kind, params) in SMALL.items()}


@pytest.mark.parametrize("restart", [30, 8])
@pytest.mark.parametrize("name", list(SMALL))
def test_fgmres_matches_oracle(orc, ctx, cases, name, restart):
    say("fgmres", name, restart)
    c = cases[name]
    b = W.rhs(c.A.n, 0)
    x0 = W.rhs(c.A.n, 3) * 0.01
    k_ref, x_ref, h_ref = orc.fgmres(c.A, c.Ls, c.Us, c.dinv, b, x0, m=restart, max_iters=400, tol=1e-8)
    assert k_ref < 400
    x = dev(x0)
    k, hist = ctx.fgmres(c.Ad, c.F, dev(b), x, restart=restart, max_iters=400, tol=1e-8)
    assert k == k_ref, f"{name}: GPU {k} steps, oracle {k_ref}"
    np.testing.assert_allclose(hist, h_ref, rtol=1e-6, atol=0)
    assert_close(host(x), x_ref, 1e-7, f"fgmres {name}")
    true = np.linalg.norm(orc.residual(c.A, b, host(x))) / np.linalg.norm(b)
    assert true < 1.01e-8


@pytest.mark.parametrize("name", ["poisson17", "aniso11_ilut"])
def test_fgmres_mixed_preconditioner(orc, ctx, cases, name):
    """The FP32-inner preconditioner inside FGMRES: converges to the same
    tolerance in about the same number of steps as the FP64 one."""
    say("fgmres mixed", name)
    c = cases[name]
    b = W.rhs(c.A.n, 0)
    k_ref, _, _ = orc.fgmres(c.A, c.Ls, c.Us, c.dinv, b, np.zeros(c.A.n), m=30, max_iters=400, tol=1e-8)
    x = dev(np.zeros(c.A.n))
    k, hist = ctx.fgmres(c.Ad, c.F, dev(b), x, restart=30, max_iters=400, tol=1e-8, mixed=True)
    assert abs(k - k_ref) <= 1
    true = np.linalg.norm(orc.residual(c.A, b, host(x))) / np.linalg.norm(b)
    assert true < 1.01e-8


def test_fgmres_exact_preconditioner(orc, B, ctx):
    A = W.tridiag(300)
    Ls, U = orc.ilu0(A)
    F = ctx.ilu_scale_factors(B.Csr.from_host(Ls), B.Csr.from_host(U))
    b = W.rhs(A.n, 1)
    x = dev(np.zeros(A.n))
    k, hist = ctx.fgmres(B.Csr.from_host(A), F, dev(b), x, restart=10, max_iters=10, tol=1e-10, m_L=300, m_U=300)
    assert k == 1
    assert_close(host(x), np.linalg.solve(A.to_dense(), b), 1e-11, "exact preconditioner")


def test_already_converged_and_errors(orc, B, ctx, cases):
    c = cases["poisson17"]
    xs = W.rhs(c.A.n, 5)
    b = orc.spmv(c.A, xs)
    x = dev(xs)
    k, hist = ctx.fgmres(c.Ad, c.F, dev(b), x, tol=1e-8)
    assert k == 0
    np.testing.assert_array_equal(host(x), xs)
    with pytest.raises(B.SiluError) as e:
        ctx.fgmres(c.Ad, c.F, dev(b), dev(xs), restart=0)
    assert e.value.status == -1
    G = ctx.gs_split(c.Ad)
    with pytest.raises(B.SiluError) as e:
        ctx.fgmres(c.Ad, G, dev(b), dev(xs))
    assert e.value.status == -8


@pytest.mark.parametrize("kernel", [None, "sliced32", "stream", "stream32"])
@pytest.mark.parametrize("name", list(SMALL))
def test_spmv_bitwise(orc, ctx, cases, name, kernel):
    c = cases[name]
    v = W.rhs(c.A.n, 9)
    np.testing.assert_array_equal(host(ctx.spmv(c.Ad, dev(v), kernel=kernel)), orc.spmv(c.A, v))


def test_dot_and_norm_estimate(orc, B, ctx, cases):
    rng = np.random.default_rng(2)
    for n in (1, 1000, 1 << 20, (1 << 20) + 77):
        a, b = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
        got = ctx.dot(dev(a), dev(b))
        assert got == pytest.approx(float(np.dot(a, b)), rel=1e-12, abs=1e-12)
    c = cases["poisson17"]
    est = ctx.norm2_estimate(c.Ad, iters=300)
    lam = 6.0 + 6.0 * np.cos(np.pi / 18)  # largest eigenvalue of the 7-point Dirichlet Laplacian, N = 17
    assert est == pytest.approx(lam, rel=2e-3)
    x = W.rhs(c.A.n, 4)
    b = W.rhs(c.A.n, 5)
    r = orc.residual(c.A, b, x)
    ref = np.linalg.norm(r) / (np.linalg.norm(b) + lam * np.linalg.norm(x))
    assert ctx.nrbe(c.Ad, dev(b), dev(x), lam) == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("name", list(SMALL))
def test_zero_guess_flag(ctx, cases, name):
    """With x = 0 the zero-guess smoother skips the first residual and gives
    the same bits."""
    c = cases[name]
    b = dev(W.rhs(c.A.n, 6))
    for mixed in (False, True):
        x1, x2 = dev(np.zeros(c.A.n)), dev(np.zeros(c.A.n))
        ctx.ilu_smooth(c.Ad, c.F, b, x1, 2, 3, 3, mixed=mixed)
        ctx.ilu_smooth(c.Ad, c.F, b, x2, 2, 3, 3, mixed=mixed, zero_guess=True)
        np.testing.assert_array_equal(host(x1), host(x2))


@pytest.mark.parametrize("name", ["perm9", "vardens13_ilu1"])
@pytest.mark.parametrize("mixed", [False, True])
def test_fgmres_on_relabeled_copies(orc, ctx, cases, name, mixed):
    """SILU_REORDER: the whole solve runs in the relabeled order.  Every
    product and sweep keeps its bits (rows keep their storage order), the dot
    products sum in another order, so the run equals the given-order run to
    the Krylov tolerance (same steps, estimates to 1e-6, solution to 1e-7 of
    its max norm); in FP64 also the oracle's."""
    c = cases[name]
    bh = W.rhs(c.A.n, 3)
    b = dev(bh)
    x1, x2 = torch.zeros_like(b), torch.zeros_like(b)
    k1, h1 = ctx.fgmres(c.Ad, c.F, b, x1, restart=8, max_iters=60, tol=1e-10, mixed=mixed)
    k2, h2 = ctx.fgmres(c.Ad, c.F, b, x2, restart=8, max_iters=60, tol=1e-10, mixed=mixed, reorder=True)
    assert k1 == k2
    np.testing.assert_allclose(h2, h1, rtol=1e-6, atol=1e-15 * h1[0])
    assert_close(host(x2), host(x1), 1e-7, f"fgmres relabeled {name}")
    if not mixed:
        k_ref, x_ref, h_ref = orc.fgmres(c.A, c.Ls, c.Us, c.dinv, bh, np.zeros(c.A.n), m=8, max_iters=60, tol=1e-10)
        assert k2 == k_ref
        np.testing.assert_allclose(h2, h_ref, rtol=1e-6, atol=1e-15 * h_ref[0])
        assert_close(host(x2), x_ref, 1e-7, f"fgmres relabeled vs oracle {name}")


def test_fgmres_relabeled_nrbe_and_initial_guess(orc, ctx, cases):
    """The relabeled solve with a nonzero initial guess (permuted in with b) and
    the NRBE rule, against the oracle; and a guess that already satisfies the
    rule comes back unchanged."""
    c = cases["perm9"]
    na = _norm2_host(c.A)
    bh, x0 = W.rhs(c.A.n, 0), W.rhs(c.A.n, 3) * 0.01
    k_ref, x_ref, h_ref = orc.fgmres(c.A, c.Ls, c.Us, c.dinv, bh, x0, m=30, max_iters=200, tol=1e-12, norm_a=na)
    x = dev(x0)
    k, hist = ctx.fgmres(c.Ad, c.F, dev(bh), x, restart=30, max_iters=200, tol=1e-12, norm_a=na, reorder=True)
    assert k == k_ref
    np.testing.assert_allclose(hist, h_ref, rtol=1e-6, atol=1e-15 * h_ref[0])
    assert_close(host(x), x_ref, 1e-7, "fgmres relabeled nrbe")
    xs = W.rhs(c.A.n, 5)
    bs = orc.spmv(c.A, xs)
    x = dev(xs)
    k, _ = ctx.fgmres(c.Ad, c.F, dev(bs), x, tol=1e-8, reorder=True)
    assert k == 0
    np.testing.assert_array_equal(host(x), xs)


# ---- FGMRES stopped on the norm-wise relative backward error (eq. nbre) ----

def _norm2_host(A):
    """||A||_2 on the host (largest singular value, ARPACK from a fixed start)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla

    Ah = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))
    return float(sla.svds(Ah, k=1, v0=np.ones(A.n), return_singular_vectors=False)[0])


@pytest.mark.parametrize("restart", [30, 8])
@pytest.mark.parametrize("name", list(SMALL))
def test_fgmres_nrbe_matches_oracle(orc, ctx, cases, name, restart):
    """Same steps, estimates and solution as the oracle, whose ||x_j|| comes from
    the iterate formed after every step (the library's from the Gram matrix of
    the directions).  tol = 1e-12: every estimate of these runs is at least 7%
    away from it, far more than the two sides' rounding differences."""
    say("fgmres nrbe", name, restart)
    c = cases[name]
    na = _norm2_host(c.A)
    b = W.rhs(c.A.n, 0)
    x0 = W.rhs(c.A.n, 3) * 0.01
    k_ref, x_ref, h_ref = orc.fgmres(c.A, c.Ls, c.Us, c.dinv, b, x0, m=restart, max_iters=400, tol=1e-12,
                                     norm_a=na)
    assert 0 < k_ref < 400
    x = dev(x0)
    k, hist = ctx.fgmres(c.Ad, c.F, dev(b), x, restart=restart, max_iters=400, tol=1e-12, norm_a=na)
    assert k == k_ref, f"{name}: GPU {k} steps, oracle {k_ref}"
    # the Arnoldi residual |g_j| carries an absolute rounding error of order
    # eps ||r_0|| on either side (not one relative to |g_j|), which matters once
    # the estimates fall four decades below those of the relres runs: hence
    # the absolute term, 1e-15 of the first estimate
    np.testing.assert_allclose(hist, h_ref, rtol=1e-6, atol=1e-15 * h_ref[0])
    assert_close(host(x), x_ref, 1e-7, f"fgmres nrbe {name}")
    xh = host(x)
    true = np.linalg.norm(orc.residual(c.A, b, xh)) / (np.linalg.norm(b) + na * np.linalg.norm(xh))
    assert true < 1.01e-12


def test_fgmres_nrbe_with_zero_norm_is_fgmres(ctx, cases):
    """norm_a = 0 turns eq. nbre into eq. relres: the same run bit for bit."""
    c = cases["vardens13_ilu1"]
    b = dev(W.rhs(c.A.n, 1))
    x1, x2 = torch.zeros_like(b), torch.zeros_like(b)
    k1, h1 = ctx.fgmres(c.Ad, c.F, b, x1, restart=8, max_iters=50, tol=1e-9)
    k2, h2 = ctx.fgmres(c.Ad, c.F, b, x2, restart=8, max_iters=50, tol=1e-9, norm_a=0.0)
    assert k1 == k2
    np.testing.assert_array_equal(h1, h2)
    np.testing.assert_array_equal(host(x1), host(x2))


def test_norm2_estimate_follows_its_definition(B, ctx, cases):
    """The power iteration of silu_norm2_estimate from the binding's start
    vector, repeated on the host with the same start: same value to rounding
    (a non-symmetric operator, so it is not ||A||_2 itself)."""
    import scipy.sparse as sp

    c = cases["perm9"]
    A = c.A
    Ah = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))
    g = torch.Generator(device="cpu").manual_seed(4)
    v = (torch.rand(A.n, generator=g, dtype=torch.float64) - 0.5).numpy()
    v = v / np.linalg.norm(v)
    lam = 0.0
    for _ in range(7):
        w = Ah @ v
        lam = np.linalg.norm(w)
        v = w / lam
    assert ctx.norm2_estimate(c.Ad, iters=7, seed=4) == pytest.approx(lam, rel=1e-12)


def test_nrbe_and_norm_errors(B, ctx, cases):
    import ctypes as C

    c = cases["poisson17"]
    b = dev(W.rhs(c.A.n, 0))
    with pytest.raises(B.SiluError) as e:
        ctx.nrbe(c.Ad, b, b.clone(), -1.0)
    assert e.value.status == -1
    with pytest.raises(B.SiluError) as e:
        ctx.fgmres(c.Ad, c.F, b, torch.zeros_like(b), norm_a=float("inf"))
    assert e.value.status == -1
    with pytest.raises(B.SiluError) as e:
        ctx.norm2_estimate(c.Ad, iters=0)
    assert e.value.status == -1
    # a zero start vector has no direction
    ws = ctx._aux_ws(c.A.n)
    z = torch.zeros_like(b)
    out = C.c_double()
    Ac = c.Ad.c()
    st = B._lib.silu_norm2_estimate(ctx._h, C.byref(Ac), C.c_void_p(z.data_ptr()), 5, C.byref(out),
                                    C.c_void_p(ws.data_ptr()), ws.numel())
    assert st == -1
    st = B._lib.silu_nrbe(ctx._h, C.byref(Ac), C.c_void_p(b.data_ptr()), C.c_void_p(b.data_ptr()), 1.0,
                          C.byref(out), C.c_void_p(ws.data_ptr()), 100)
    assert st == -6  # workspace too small (SILU_ERR_NOMEM)


@pytest.mark.parametrize("case", ["one_row", "restart1", "no_steps"])
def test_fgmres_nrbe_edge_cases(orc, B, ctx, case):
    """A 1 x 1 system (exact after one step, estimate 0), restart = 1 (every
    step a restart, so ||x_0|| is refreshed each time) and max_iters = 0 (only
    the initial estimate): against the oracle."""
    if case == "one_row":
        A, m, iters, bh = W.CSR.from_dense(np.array([[4.0]])), 1, 5, np.array([2.0])
    else:
        A = W.poisson7(5)
        m, iters, bh = (1, 40, W.rhs(A.n, 0)) if case == "restart1" else (5, 0, W.rhs(A.n, 0))
    Ls, U = orc.ilu0(A)
    _, dinv, Us = orc.scale_rows(U)
    F = ctx.ilu_scale_factors(B.Csr.from_host(Ls), B.Csr.from_host(U))
    Ad = B.Csr.from_host(A)
    na = 4.0 if case == "one_row" else _norm2_host(A)
    x0 = np.zeros(A.n) if case == "one_row" else W.rhs(A.n, 2) * 0.01
    k_ref, x_ref, h_ref = orc.fgmres(A, Ls, Us, dinv, bh, x0, m=m, max_iters=iters, tol=1e-12, norm_a=na)
    x = dev(x0)
    k, hist = ctx.fgmres(Ad, F, dev(bh), x, restart=m, max_iters=iters, tol=1e-12, norm_a=na)
    assert k == k_ref
    np.testing.assert_allclose(hist, h_ref, rtol=1e-6, atol=1e-15 * h_ref[0])
    assert_close(host(x), x_ref, 1e-7, f"fgmres nrbe {case}")
    if case == "one_row":
        assert ctx.norm2_estimate(Ad, iters=3) == pytest.approx(4.0, rel=1e-15)
        assert ctx.nrbe(Ad, dev(bh), x, 4.0) == 0.0
