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
def test_fgmres_with_relabeled_preconditioner(ctx, cases, name, mixed):
    """SILU_REORDER inside FGMRES: every preconditioner application is bit for
    bit the plain one, so the whole run is too."""
    c = cases[name]
    b = dev(W.rhs(c.A.n, 3))
    x1, x2 = torch.zeros_like(b), torch.zeros_like(b)
    k1, h1 = ctx.fgmres(c.Ad, c.F, b, x1, restart=8, max_iters=60, tol=1e-10, mixed=mixed)
    k2, h2 = ctx.fgmres(c.Ad, c.F, b, x2, restart=8, max_iters=60, tol=1e-10, mixed=mixed, reorder=True)
    assert k1 == k2
    np.testing.assert_array_equal(h1, h2)
    np.testing.assert_array_equal(host(x1), host(x2))
