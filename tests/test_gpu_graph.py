"""GPU tests of SILU_GRAPH: a smoother call recorded once into a hipGraph and
replayed.  Every replay, with the program's own eager work and
synchronizations in between, must equal the plain-launch call bit for bit
(and so the oracle); releasing a matrix, or changing its values in place,
must drop the recording so that the next call reads the current data."""
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
    (1, 1, 1, False, False, None),  # residual fused with D^{-1}, then the axpy
    (1, 1, 3, False, False, None),
    (2, 3, 2, False, False, "stream"),
]


def _eager_other_work():
    junk = torch.randn(1 << 14, device="cuda").cumsum(0)
    torch.cuda.synchronize()
    assert torch.isfinite(junk).all()


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("variant", VARIANTS, ids=lambda v: "o{}_L{}_U{}{}{}{}".format(
    v[0], v[1], v[2], "_mixed" if v[3] else "", "_zero" if v[4] else "", f"_{v[5]}" if v[5] else ""))
def test_replays_equal_plain_calls(orc, B, ctx, cases, name, variant):
    outer, mL, mU, mixed, zero, kernel = variant
    say("graph", name, variant)
    c = cases[name]
    n = c.A.n
    b = W.rhs(n, 5)
    x0 = np.zeros(n) if zero else W.rhs(n, 6)
    bd, ws = dev(b), ctx.workspace(n)
    xe = dev(x0)
    ctx.ilu_smooth(c.Ad, c.F, bd, xe, outer, mL, mU, mixed=mixed, zero_guess=zero, kernel=kernel, ws=ws)
    ref = host(xe)
    if not mixed:
        np.testing.assert_array_equal(ref, orc.smooth(c.A, c.Ls, c.Us, c.dinv, b, x0, outer, mL, mU))
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    for rep in range(4):  # the first call records, the others replay
        x.copy_(dev(x0))
        ctx.ilu_smooth(c.Ad, c.F, bd, x, outer, mL, mU, mixed=mixed, zero_guess=zero, kernel=kernel, ws=ws,
                       record=True)
        np.testing.assert_array_equal(host(x), ref)
        _eager_other_work()
        xo = dev(x0)  # a plain call on other buffers between replays
        ctx.ilu_smooth(c.Ad, c.F, bd, xo, outer, mL, mU, mixed=mixed, zero_guess=zero, kernel=kernel, ws=ws)
        np.testing.assert_array_equal(host(xo), ref)


def test_rowcol_and_unscaled_replays(orc, B, ctx, cases):
    c = cases["vardens13_ilu1"]
    n = c.A.n
    b, x0 = W.rhs(n, 1), W.rhs(n, 2)
    bd, ws = dev(b), ctx.workspace(n)
    for F in (ctx.ilu_scale_factors_rowcol(c.Ld, c.Ud, 5), ctx.ilu_scale_factors(c.Ld, c.Ud, scale=False)):
        xe = dev(x0)
        ctx.ilu_smooth(c.Ad, F, bd, xe, 2, 3, 3, ws=ws)
        ref = host(xe)
        x = torch.empty(n, dtype=torch.float64, device="cuda")
        for rep in range(3):
            x.copy_(dev(x0))
            ctx.ilu_smooth(c.Ad, F, bd, x, 2, 3, 3, ws=ws, record=True)
            np.testing.assert_array_equal(host(x), ref)
            _eager_other_work()


def test_recording_dropped_on_release_and_value_change(orc, B, ctx):
    """Values changed in place: the binding releases the matrix, which drops
    every recording, so the replay path re-records on the new values."""
    say("graph: value change")
    A = W.vardens7(11, seed_rho=3)
    Ls, U = orc.ilu0(A)
    d, dinv, Us = orc.scale_rows(U)
    Ad, Ld, Ud = B.Csr.from_host(A), B.Csr.from_host(Ls), B.Csr.from_host(U)
    F = ctx.ilu_scale_factors(Ld, Ud)
    b = W.rhs(A.n, 0)
    bd, ws = dev(b), ctx.workspace(A.n)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    for _ in range(2):
        x.zero_()
        ctx.ilu_smooth(Ad, F, bd, x, 1, 3, 3, ws=ws, record=True)
        np.testing.assert_array_equal(host(x), orc.smooth(A, Ls, Us, dinv, b, np.zeros(A.n), 1, 3, 3))
    Ad.val.mul_(2.0)
    A2 = W.CSR(A.n, A.row_ptr, A.col, A.val * 2.0)
    for _ in range(3):
        x.zero_()
        ctx.ilu_smooth(Ad, F, bd, x, 1, 3, 3, ws=ws, record=True)
        np.testing.assert_array_equal(host(x), orc.smooth(A2, Ls, Us, dinv, b, np.zeros(A.n), 1, 3, 3))
        _eager_other_work()


def test_replay_stats_and_flags(orc, B, ctx, cases):
    """A replay is one timed launch credited with the recorded sequence's bytes;
    CHECK_FINITE still scans x after a replay."""
    c = cases["poisson17"]
    n = c.A.n
    bd, ws = dev(W.rhs(n, 0)), ctx.workspace(n)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    ctx.stats_reset()
    ctx.set_timing(True)
    ctx.ilu_smooth(c.Ad, c.F, bd, x, 1, 3, 3, ws=ws)
    plain = ctx.stats()
    ctx.stats_reset()
    x.zero_()
    ctx.ilu_smooth(c.Ad, c.F, bd, x, 1, 3, 3, ws=ws, record=True)  # records (plain launches run)
    x.zero_()
    ctx.stats_reset()
    ctx.ilu_smooth(c.Ad, c.F, bd, x, 1, 3, 3, ws=ws, record=True, check_finite=True)  # replays
    rep = ctx.stats()
    ctx.set_timing(False)
    assert rep["smooth_graph"]["launches"] == 1
    want = sum(v["bytes"] for v in plain.values() if v["launches"])
    assert rep["smooth_graph"]["bytes"] == pytest.approx(want, rel=1e-12)
    want_l = sum(v["layout_bytes"] for v in plain.values() if v["launches"])
    assert rep["smooth_graph"]["layout_bytes"] == pytest.approx(want_l, rel=1e-12)
