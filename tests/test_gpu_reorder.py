"""GPU tests of SILU_REORDER: the sweeps on locality-relabeled copies of A and
the factors give the plain call's result bit for bit (each row keeps its
entries in their original order), in every form of the smoother; the copies
follow the matrices' lifetime and values."""
import numpy as np
import pytest
import torch

from paper_2111_09512_amd import workloads as W
from tests.gpu_common import Case, dev, host, need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    need_gpu()
    from paper_2111_09512_amd import binding

    return binding


@pytest.fixture(scope="module")
def ctx(B):
    return B.Context()


SMALL = {
    "poisson17": (lambda: W.poisson7(17), "ilu0", {}),
    "vardens13_ilu1": (lambda: W.vardens7(13), "iluk", {"k": 1}),
    "aniso11_ilut": (lambda: W.aniso27(11), "ilut", {"tau": 1e-3, "p": 20}),
    "perm9": (lambda: W.permuted_longrange7(9, seed=1), "ilu0", {}),
    "perm17": (lambda: W.permuted_longrange7(17, seed=2), "ilu0", {}),
}


@pytest.fixture(scope="module")
def cases(orc, B, ctx):
    return {name: Case(orc, B, ctx, make(), kind, params, fp32=True) for name, (make, kind, params) in SMALL.items()}


# (outer, m_L, m_U, mixed, zero_guess, kernel)
VARIANTS = [
    (1, 3, 3, False, False, None),
    (2, 4, 4, False, False, None),
    (2, 3, 3, True, False, None),
    (1, 3, 3, False, True, None),
    (1, 1, 1, False, False, None),
    (2, 2, 3, True, True, None),
    (1, 3, 3, False, False, "stream"),
    (1, 3, 3, True, False, "stream"),
]


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("variant", VARIANTS, ids=lambda v: "o{}_L{}_U{}{}{}{}".format(
    v[0], v[1], v[2], "_mixed" if v[3] else "", "_zero" if v[4] else "", f"_{v[5]}" if v[5] else ""))
def test_reordered_equals_plain(orc, B, ctx, cases, name, variant):
    outer, mL, mU, mixed, zero, kernel = variant
    say("reorder", name, variant)
    c = cases[name]
    n = c.A.n
    b = W.rhs(n, 11)
    x0 = np.zeros(n) if zero else W.rhs(n, 12)
    bd = dev(b)
    xp = dev(x0)
    ctx.ilu_smooth(c.Ad, c.F, bd, xp, outer, mL, mU, mixed=mixed, zero_guess=zero, kernel=kernel)
    ref = host(xp)
    if not mixed:
        np.testing.assert_array_equal(ref, orc.smooth(c.A, c.Ls, c.Us, c.dinv, b, x0, outer, mL, mU))
    for rep in range(2):  # built on the first call, cached after
        xr = dev(x0)
        ctx.ilu_smooth(c.Ad, c.F, bd, xr, outer, mL, mU, mixed=mixed, zero_guess=zero, kernel=kernel, reorder=True)
        np.testing.assert_array_equal(host(xr), ref)


def test_rowcol_unscaled_graph_and_direct(orc, B, ctx, cases):
    c = cases["perm17"]
    n = c.A.n
    b, x0 = W.rhs(n, 1), W.rhs(n, 2)
    bd = dev(b)
    for F in (ctx.ilu_scale_factors_rowcol(c.Ld, c.Ud, 5), ctx.ilu_scale_factors(c.Ld, c.Ud, scale=False)):
        xp = dev(x0)
        ctx.ilu_smooth(c.Ad, F, bd, xp, 2, 3, 3)
        xr = dev(x0)
        ctx.ilu_smooth(c.Ad, F, bd, xr, 2, 3, 3, reorder=True, check_finite=F.scaled != 0)
        np.testing.assert_array_equal(host(xr), host(xp))
    # recorded into a hipGraph together with the permutations in and out
    F = ctx.ilu_scale_factors(c.Ld, c.Ud, fp32=True)
    xp = dev(x0)
    ctx.ilu_smooth(c.Ad, F, bd, xp, 1, 3, 3)
    ref = host(xp)
    ws = ctx.workspace(n, B.SILU_REORDER)
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    for rep in range(3):
        x.copy_(dev(x0))
        ctx.ilu_smooth(c.Ad, F, bd, x, 1, 3, 3, reorder=True, record=True, ws=ws)
        np.testing.assert_array_equal(host(x), ref)
        junk = torch.randn(4096, device="cuda").cumsum(0)
        torch.cuda.synchronize()
        assert torch.isfinite(junk).all()
    with pytest.raises(B.SiluError) as e:
        ctx.ilu_smooth(c.Ad, F, bd, dev(x0), 1, 3, 3, reorder=True, direct=True)
    assert e.value.status == -8
    with pytest.raises(B.SiluError) as e:  # the plain workspace is two vectors short
        short = torch.empty(ctx.workspace_size(n), dtype=torch.uint8, device="cuda")
        ctx.ilu_smooth(c.Ad, F, bd, dev(x0), 1, 3, 3, reorder=True, ws=short)
    assert e.value.status == -6


def test_values_changed_in_place(orc, B, ctx):
    """The relabeled copies hold values: an in-place change of A is seen."""
    say("reorder: values changed in place")
    A = W.permuted_longrange7(8, seed=4)
    Ls, U = orc.ilu0(A)
    d, dinv, Us = orc.scale_rows(U)
    Ad, Ld, Ud = B.Csr.from_host(A), B.Csr.from_host(Ls), B.Csr.from_host(U)
    F = ctx.ilu_scale_factors(Ld, Ud)
    b = W.rhs(A.n, 0)
    x = dev(np.zeros(A.n))
    ctx.ilu_smooth(Ad, F, dev(b), x, 1, 3, 3, reorder=True)
    np.testing.assert_array_equal(host(x), orc.smooth(A, Ls, Us, dinv, b, np.zeros(A.n), 1, 3, 3))
    Ad.val.mul_(2.0)
    A2 = W.CSR(A.n, A.row_ptr, A.col, A.val * 2.0)
    x = dev(np.zeros(A.n))
    ctx.ilu_smooth(Ad, F, dev(b), x, 1, 3, 3, reorder=True)
    np.testing.assert_array_equal(host(x), orc.smooth(A2, Ls, Us, dinv, b, np.zeros(A.n), 1, 3, 3))


@pytest.mark.parametrize("name", ["perm9", "perm17", "aniso11_ilut"])
def test_relabeled_vectors_equal_plain(orc, B, ctx, cases, name):
    """b and x moved into the copies' order once (silu_reorder_vectors), several
    smoother calls with SILU_REORDER | SILU_RELABELED (no permutations inside),
    x moved back once: the same bits as the same calls in the given order, FP64
    and FP32-inner, from a zero guess too; and moving a vector in and out gives
    it back."""
    say("relabeled vectors", name)
    c = cases[name]
    n = c.A.n
    b, x0 = dev(W.rhs(n, 3)), dev(W.rhs(n, 4))
    np.testing.assert_array_equal(host(ctx.reorder_vectors(c.Ad, c.F, ctx.reorder_vectors(c.Ad, c.F, x0),
                                                           to_relabeled=False)), host(x0))
    for mixed in (False, True):
        for zero in (False, True):
            start = torch.zeros_like(x0) if zero else x0.clone()
            x = start.clone()
            for _ in range(3):
                ctx.ilu_smooth(c.Ad, c.F, b, x, 1, 3, 3, mixed=mixed, zero_guess=zero and _ == 0)
            b2 = ctx.reorder_vectors(c.Ad, c.F, b)
            x2 = ctx.reorder_vectors(c.Ad, c.F, start)
            ws = ctx.workspace(n, B.SILU_REORDER | B.SILU_RELABELED)
            for _ in range(3):
                ctx.ilu_smooth(c.Ad, c.F, b2, x2, 1, 3, 3, mixed=mixed, zero_guess=zero and _ == 0, reorder=True,
                               relabeled=True, ws=ws)
            np.testing.assert_array_equal(host(ctx.reorder_vectors(c.Ad, c.F, x2, to_relabeled=False)), host(x))
    with pytest.raises(B.SiluError):  # relabeled vectors without the relabeled copies
        ctx.ilu_smooth(c.Ad, c.F, b, x0.clone(), 1, 3, 3, relabeled=True)
