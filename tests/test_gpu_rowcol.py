"""GPU parity of the row/column scaling (Section 5.1, eq. rowcolScale): the
Ruiz set-up and the smoother on U^ = D_r U D_c, through the C-ABI, against
the oracle on the same seeded inputs.

Bars: the set-up is bit-identical (maxima are exact; every other step is one
IEEE operation in the oracle's order); FP64 smoothing 1e-12 relative and
bit-identical for the kernels that sum rows in the oracle's order; the mixed
form bit-identical to the oracle's FP32 emulation for those kernels and within
1e-5 of FP64; the direct path 1e-12."""
import numpy as np
import pytest
import torch

from paper_2111_09512_amd import workloads as W
from tests.gpu_common import F64_TOL, MIXED_TOL, assert_close, dev, host, need_gpu, say

pytestmark = pytest.mark.gpu

KERNELS = [None, "sliced16", "sliced32", "stream", "win", "stream16", "stream32", "blocked", "vector"]
RUIZ = 5

SMALL = {
    "poisson17": (lambda: W.poisson7(17), "ilu0", {}),
    "vardens13_ilu1": (lambda: W.vardens7(13), "iluk", {"k": 1}),
    "aniso11_ilut": (lambda: W.aniso27(11), "ilut", {"tau": 1e-3, "p": 20}),
    "perm9": (lambda: W.permuted_longrange7(9, seed=1), "ilu0", {}),
    "mmatrix3000": (lambda: W.random_mmatrix(3000, 0.002, seed=9), "ilu0", {}),
}


@pytest.fixture(scope="module")
def B():
    need_gpu()
    from paper_2111_09512_amd import binding

    return binding


@pytest.fixture(scope="module")
def ctx(B):
    return B.Context()


class RCCase:
    def __init__(self, orc, B, ctx, A, kind, params):
        self.A = A
        self.Ls, self.U = orc.factor(A, kind, params)
        self.dr, self.dc, self.Uh, _ = orc.scale_rowcol(self.U, RUIZ)
        self.d, self.dinv, self.Us = orc.scale_rows(self.U)
        self.Ad, self.Ld, self.Ud = B.Csr.from_host(A), B.Csr.from_host(self.Ls), B.Csr.from_host(self.U)
        self.F = ctx.ilu_scale_factors_rowcol(self.Ld, self.Ud, RUIZ, fp32=True)
        self.Frow = ctx.ilu_scale_factors(self.Ld, self.Ud)
        torch.cuda.synchronize()


@pytest.fixture(scope="module")
def cases(orc, B, ctx):
    return {name: RCCase(orc, B, ctx, make(), kind, params) for name, (make, kind, params) in SMALL.items()}


@pytest.mark.parametrize("name", list(SMALL))
def test_rowcol_factors_bitwise(cases, name):
    say("rowcol scale", name)
    c = cases[name]
    F = c.F
    assert F.scaled == 2
    np.testing.assert_array_equal(host(F.Us.row_ptr), c.Uh.row_ptr)
    np.testing.assert_array_equal(host(F.Us.col_idx), c.Uh.col)
    np.testing.assert_array_equal(host(F.dc), c.dc)
    np.testing.assert_array_equal(host(F.dinv), c.dr)
    np.testing.assert_array_equal(host(F.Us.val), c.Uh.val)
    np.testing.assert_array_equal(host(F.d), c.d)
    np.testing.assert_array_equal(host(F.Us_val32), c.Uh.val.astype(np.float32))
    np.testing.assert_array_equal(host(F.Ls_val32), c.Ls.val.astype(np.float32))


@pytest.mark.parametrize("iters", [0, 1, 12])
def test_rowcol_iteration_counts(orc, B, ctx, iters):
    say("rowcol iters", iters)
    A = W.random_mmatrix(1500, 0.004, seed=4)
    Ls, U = orc.ilu0(A)
    dr, dc, Uh, _ = orc.scale_rowcol(U, iters)
    F = ctx.ilu_scale_factors_rowcol(B.Csr.from_host(Ls), B.Csr.from_host(U), iters)
    np.testing.assert_array_equal(host(F.dc), dc)
    np.testing.assert_array_equal(host(F.dinv), dr)
    np.testing.assert_array_equal(host(F.Us.val), Uh.val)


SCHED = [(1, 3, 3), (2, 4, 4), (1, 1, 1), (1, 1, 3), (1, 3, 1), (3, 2, 5)]


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("sched", SCHED, ids=lambda s: "o%dL%dU%d" % s)
@pytest.mark.parametrize("name", list(SMALL))
def test_rowcol_smooth_f64(orc, ctx, cases, name, sched, kernel):
    outer, mL, mU = sched
    say("rowcol smooth f64", name, sched, kernel)
    c = cases[name]
    b = W.rhs(c.A.n, 0)
    x0 = W.rhs(c.A.n, 7) if outer > 1 else np.zeros(c.A.n)
    ref = orc.smooth_rowcol(c.A, c.Ls, c.Uh, c.dr, c.dc, b, x0, outer, mL, mU)
    x = dev(x0)
    ctx.ilu_smooth(c.Ad, c.F, dev(b), x, outer, mL, mU, kernel=kernel)
    got = host(x)
    assert_close(got, ref, F64_TOL, f"rowcol {name} {sched} {kernel}")
    if kernel != "vector":
        np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("kernel", [None, "vector"])
@pytest.mark.parametrize("sched", [(1, 3, 3), (1, 1, 1), (1, 2, 1), (2, 1, 4)], ids=lambda s: "o%dL%dU%d" % s)
@pytest.mark.parametrize("name", list(SMALL))
def test_rowcol_smooth_mixed(orc, ctx, cases, name, sched, kernel):
    outer, mL, mU = sched
    say("rowcol smooth mixed", name, sched, kernel)
    c = cases[name]
    b = W.rhs(c.A.n, 0)
    x0 = np.zeros(c.A.n)
    ref64 = orc.smooth_rowcol(c.A, c.Ls, c.Uh, c.dr, c.dc, b, x0, outer, mL, mU)
    ref32 = orc.smooth_rowcol(c.A, c.Ls, c.Uh, c.dr, c.dc, b, x0, outer, mL, mU, mixed=True)
    x = dev(x0)
    ctx.ilu_smooth(c.Ad, c.F, dev(b), x, outer, mL, mU, mixed=True, kernel=kernel)
    got = host(x)
    assert_close(got, ref64, MIXED_TOL, f"rowcol mixed {name} {sched}")
    if kernel != "vector":
        np.testing.assert_array_equal(got, ref32)


@pytest.mark.parametrize("name", list(SMALL))
def test_rowcol_smooth_direct(orc, ctx, cases, name):
    say("rowcol direct", name)
    c = cases[name]
    b, x0 = W.rhs(c.A.n, 0), W.rhs(c.A.n, 3)
    ref = orc.smooth_rowcol(c.A, c.Ls, c.Uh, c.dr, c.dc, b, x0, 2, 0, 0, direct=True)
    for graph in (True, False):
        x = dev(x0)
        ctx.ilu_smooth(c.Ad, c.F, dev(b), x, 2, 1, 1, direct=True, graph=graph)
        assert_close(host(x), ref, F64_TOL, f"rowcol direct {name} graph={graph}")


@pytest.mark.parametrize("name", ["mmatrix3000", "aniso11_ilut"])
def test_rowcol_equals_row_scaling(ctx, cases, name):
    """Similarity invariance on the device: the two scalings give the same x
    to rounding."""
    say("rowcol vs row", name)
    c = cases[name]
    b = W.rhs(c.A.n, 5)
    x1, x2 = dev(np.zeros(c.A.n)), dev(np.zeros(c.A.n))
    ctx.ilu_smooth(c.Ad, c.F, dev(b), x1, 2, 3, 4)
    ctx.ilu_smooth(c.Ad, c.Frow, dev(b), x2, 2, 3, 4)
    assert_close(host(x1), host(x2), 1e-11, f"rowcol vs row {name}")


def test_rowcol_serving(B, ctx, cases):
    """Served requests on row/column-scaled factors equal their lone runs."""
    say("rowcol serving")
    names = ["poisson17", "mmatrix3000", "perm9"]
    server = B.Server(ctx, arena_bytes=32 << 20, max_active=8)
    mids = [server.register(cases[nm].Ad, cases[nm].F) for nm in names]
    reqs, xs, tickets = [], [], []
    for k in range(12):
        nm = names[k % 3]
        n = cases[nm].A.n
        r = (nm, W.rhs(n, 40 + k), 1 + k % 3, [(3, 3), (1, 2), (2, 1)][k % 3])
        reqs.append(r)
        x = dev(np.zeros(n))
        xs.append(x)
        tickets.append(server.submit(mids[k % 3], dev(r[1]), x, r[2], *r[3]))
    left = set(tickets)
    while left:
        server.step()
        for t in list(left):
            if server.poll(t) == server.DONE:
                left.discard(t)
    for k, (nm, b, outer, (mL, mU)) in enumerate(reqs):
        c = cases[nm]
        x = dev(np.zeros(c.A.n))
        ctx.ilu_smooth(c.Ad, c.F, dev(b), x, outer, mL, mU)
        np.testing.assert_array_equal(host(xs[k]), host(x))
    server.close()


def test_rowcol_errors(B, ctx, cases):
    say("rowcol errors")
    c = cases["poisson17"]
    with pytest.raises(B.SiluError) as e:
        ctx.ilu_scale_factors_rowcol(c.Ld, c.Ud, 101)
    assert e.value.status == -1
    with pytest.raises(B.SiluError) as e:
        ctx.ilu_scale_factors_rowcol(c.Ld, c.Ud, -1)
    assert e.value.status == -1
    U = W.CSR.from_dense(np.array([[2.0, 1.0, 0.0], [0.0, 1.0, 3.0], [0.0, 0.0, 1.0]]))
    U.val[U.row_ptr[1]] = 0.0
    L = W.CSR.from_dense(np.zeros((3, 3)))
    with pytest.raises(B.SiluError) as e:
        ctx.ilu_scale_factors_rowcol(B.Csr.from_host(L), B.Csr.from_host(U))
    assert e.value.status == -4 and e.value.row == 1
    Fbad = B.Factors(c.F.Ls, c.F.Us, c.F.d, c.F.dinv, None, None, 2, None)  # column factors missing
    with pytest.raises(B.SiluError) as e:
        ctx.ilu_smooth(c.Ad, Fbad, dev(W.rhs(c.A.n, 0)), dev(np.zeros(c.A.n)), 1, 2, 2)
    assert e.value.status == -1
