"""GPU parity of the polynomial Gauss-Seidel smoother (Section 2's comparison
smoother) through the C-ABI against the oracle on the same seeded inputs.

Bars: the split is bit-identical (one division per entry); FP64 smoothing
1e-12 relative and bit-identical for the kernels that sum rows in the
oracle's order; the mixed form bit-identical to the oracle's FP32 emulation
for those kernels and within 1e-5 of FP64."""
import numpy as np
import pytest
import torch

from paper_2111_09512_amd import workloads as W
from tests.gpu_common import F64_TOL, MIXED_TOL, assert_close, dev, host, need_gpu, say

pytestmark = pytest.mark.gpu

KERNELS = [None, "sliced16", "sliced32", "stream", "stream32", "vector"]

SMALL = {
    "poisson17": lambda: W.poisson7(17),
    "vardens13": lambda: W.vardens7(13),
    "aniso11": lambda: W.aniso27(11),
    "perm9": lambda: W.permuted_longrange7(9, seed=1),
    "mmatrix3000": lambda: W.random_mmatrix(3000, 0.002, seed=9),
}


@pytest.fixture(scope="module")
def B():
    need_gpu()
    from paper_2111_09512_amd import binding

    return binding


@pytest.fixture(scope="module")
def ctx(B):
    return B.Context()


class GCase:
    def __init__(self, orc, B, ctx, A):
        self.A = A
        self.Gs, self.dinv = orc.gs_split(A)
        self.Ad = B.Csr.from_host(A)
        self.G = ctx.gs_split(self.Ad, fp32=True)
        torch.cuda.synchronize()


@pytest.fixture(scope="module")
def cases(orc, B, ctx):
    return {name: GCase(orc, B, ctx, make()) for name, make in SMALL.items()}


@pytest.mark.parametrize("name", list(SMALL))
def test_split_bitwise(cases, name):
    say("gs split", name)
    c = cases[name]
    np.testing.assert_array_equal(host(c.G.Ls.row_ptr), c.Gs.row_ptr)
    np.testing.assert_array_equal(host(c.G.Ls.col_idx), c.Gs.col)
    np.testing.assert_array_equal(host(c.G.Ls.val), c.Gs.val)
    np.testing.assert_array_equal(host(c.G.dinv), c.dinv)
    np.testing.assert_array_equal(host(c.G.Ls_val32), c.Gs.val.astype(np.float32))
    assert c.G.scaled == 3


SCHED = [(1, 1), (1, 2), (1, 4), (2, 3), (3, 5)]


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("sched", SCHED, ids=lambda s: "o%dt%d" % s)
@pytest.mark.parametrize("name", list(SMALL))
def test_gs_smooth_f64(orc, ctx, cases, name, sched, kernel):
    outer, terms = sched
    say("gs smooth f64", name, sched, kernel)
    c = cases[name]
    b = W.rhs(c.A.n, 0)
    x0 = W.rhs(c.A.n, 7) if outer > 1 else np.zeros(c.A.n)
    ref = orc.gs_smooth(c.A, c.Gs, c.dinv, b, x0, outer, terms)
    x = dev(x0)
    ctx.gs_smooth(c.Ad, c.G, dev(b), x, outer, terms, kernel=kernel)
    got = host(x)
    assert_close(got, ref, F64_TOL, f"gs {name} {sched} {kernel}")
    if kernel != "vector":
        np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("kernel", [None, "stream", "vector"])
@pytest.mark.parametrize("sched", [(1, 1), (1, 3), (2, 4)], ids=lambda s: "o%dt%d" % s)
@pytest.mark.parametrize("name", list(SMALL))
def test_gs_smooth_mixed(orc, ctx, cases, name, sched, kernel):
    outer, terms = sched
    say("gs smooth mixed", name, sched, kernel)
    c = cases[name]
    b = W.rhs(c.A.n, 0)
    ref64 = orc.gs_smooth(c.A, c.Gs, c.dinv, b, np.zeros(c.A.n), outer, terms)
    ref32 = orc.gs_smooth(c.A, c.Gs, c.dinv, b, np.zeros(c.A.n), outer, terms, mixed=True)
    x = dev(np.zeros(c.A.n))
    ctx.gs_smooth(c.Ad, c.G, dev(b), x, outer, terms, mixed=True, kernel=kernel)
    got = host(x)
    assert_close(got, ref64, MIXED_TOL, f"gs mixed {name} {sched}")
    if kernel != "vector":
        np.testing.assert_array_equal(got, ref32)


def test_gs_exact_at_depth(orc, B, ctx, cases):
    """With depth(L) terms one step is the exact Gauss-Seidel update."""
    say("gs exact at depth")
    c = cases["poisson17"]
    depth = orc.levels(c.Gs, "L")[1]
    b = W.rhs(c.A.n, 2)
    x = dev(np.zeros(c.A.n))
    ctx.gs_smooth(c.Ad, c.G, dev(b), x, 1, depth)
    keep = c.A.col <= np.repeat(np.arange(c.A.n), np.diff(c.A.row_ptr))  # tril(A)
    rp = np.concatenate([[0], np.cumsum(np.add.reduceat(keep, c.A.row_ptr[:-1]))]).astype(np.int32)
    T = W.CSR(c.A.n, rp, c.A.col[keep].copy(), c.A.val[keep].copy())
    ref = orc.trisolve(T, "L", False, b)
    assert_close(host(x), ref, 1e-12, "gs exact")


def test_gs_errors(B, ctx, cases):
    say("gs errors")
    c = cases["poisson17"]
    A = W.CSR.from_dense(np.array([[2.0, 0.0, 0.0], [1.0, 0.0, 1.0], [0.0, 1.0, 2.0]]))
    A.val[:] = [2.0, 1.0, 1.0, 1.0, 2.0]  # row 1 stores no diagonal
    with pytest.raises(B.SiluError) as e:
        ctx.gs_split(B.Csr.from_host(A))
    assert e.value.status == -3 and e.value.row == 1
    Z = W.CSR.from_dense(np.array([[2.0, 1.0], [1.0, 3.0]]))
    Z.val[3] = 0.0
    with pytest.raises(B.SiluError) as e:
        ctx.gs_split(B.Csr.from_host(Z))
    assert e.value.status == -4 and e.value.row == 1
    b, x = dev(W.rhs(c.A.n, 0)), dev(np.zeros(c.A.n))
    with pytest.raises(B.SiluError) as e:
        ctx.gs_smooth(c.Ad, c.G, b, x, 1, 0)
    assert e.value.status == -1
    n = c.A.n
    eye = W.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))
    F = ctx.ilu_scale_factors(c.G.Ls, B.Csr.from_host(eye))
    with pytest.raises(B.SiluError) as e:  # ILU factors are not a Gauss-Seidel split
        ctx.gs_smooth(c.Ad, F, b, x, 1, 2)
    assert e.value.status == -1


@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("name", ["perm9", "poisson17", "mmatrix3000"])
def test_gs_smooth_relabeled(orc, ctx, cases, name, mixed):
    """SILU_REORDER: the Gauss-Seidel smoother on relabeled copies equals the
    oracle (its emulation for the mixed form) bit for bit."""
    c = cases[name]
    b = W.rhs(c.A.n, 0)
    x0 = W.rhs(c.A.n, 7)
    ref = orc.gs_smooth(c.A, c.Gs, c.dinv, b, x0, 2, 3, mixed=mixed)
    for rep in range(2):
        x = dev(x0)
        ctx.gs_smooth(c.Ad, c.G, dev(b), x, 2, 3, mixed=mixed, reorder=True)
        np.testing.assert_array_equal(host(x), ref)
