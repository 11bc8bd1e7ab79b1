"""The no-allocation entry point (ilu_smooth_noalloc) against ilu_smooth2 on
the same inputs: bit for bit, FP64 and FP32-inner, with the sweeps reading
layouts a plain call cached and with none cached (the CSR arrays directly),
two calls in a row (the second on a smaller matrix, so the scratch array holds
the first call's data when the second starts), and sizes beyond the scratch
array refused."""
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


def test_noalloc_equals_plain_two_calls(orc, B):
    say("no-allocation entry point")
    ctx = B.Context()
    big = Case(orc, B, ctx, W.aniso27(23), "ilut", {"tau": 1e-3, "p": 20}, fp32=True)
    small = Case(orc, B, ctx, W.permuted_longrange7(11, seed=3), "ilu0", {}, fp32=True)
    for c, cached in ((big, True), (small, False)):
        n = c.A.n
        b, x0 = dev(W.rhs(n, 5)), dev(W.rhs(n, 6))
        for mixed in (False, True):
            for zero in (False, True):
                start = torch.zeros_like(x0) if zero else x0
                if cached:  # a plain call first: its cached layouts are read by the no-allocation call
                    want = ctx.ilu_smooth(c.Ad, c.F, b, start.clone(), 2, 3, 4, mixed=mixed, zero_guess=zero)
                got = ctx.ilu_smooth_noalloc(c.Ad, c.F, b, start.clone(), 2, 3, 4, mixed=mixed, zero_guess=zero)
                if not cached:  # the no-allocation call ran first, on the CSR arrays
                    want = ctx.ilu_smooth(c.Ad, c.F, b, start.clone(), 2, 3, 4, mixed=mixed, zero_guess=zero)
                np.testing.assert_array_equal(host(got), host(want))
                ref = (orc.smooth_mixed if mixed else orc.smooth)(c.A, c.Ls, c.Us, c.dinv, W.rhs(n, 5),
                                                                  host(start), 2, 3, 4)
                np.testing.assert_array_equal(host(got), ref)
    ctx.close()


def test_noalloc_refuses(B, orc):
    ctx = B.Context()
    c = Case(orc, B, ctx, W.poisson7(6), "ilu0", {}, fp32=True)
    b, x = dev(W.rhs(c.A.n, 1)), dev(np.zeros(c.A.n))
    with pytest.raises(B.SiluError) as e:  # a flag that would build or allocate
        ctx.ilu_smooth_noalloc(c.Ad, c.F, b, x, 1, 3, 3, kernel="blocked")
    assert e.value.status == -1
    # more rows than the scratch array holds: refused before anything runs
    n = 2 * 2**21
    A = B.Csr(torch.zeros(n + 1, dtype=torch.int32, device="cuda"), torch.zeros(1, dtype=torch.int32, device="cuda"),
              torch.zeros(1, dtype=torch.float64, device="cuda"))
    big_b = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(B.SiluError) as e:
        ctx.ilu_smooth_noalloc(A, c.F, big_b, big_b.clone(), 1, 3, 3)
    assert e.value.status == -6
    ctx.close()
