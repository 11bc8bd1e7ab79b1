"""GPU parity of ILU(0) by synchronous fixed-point sweeps (Section 7's
planned GPU factorization) against the oracle: every sweep count gives the
oracle's factors bit for bit (the same products subtracted in the same
order), the standstill is the row-wise ILU(0), and the device-computed
factors drive the smoother to the oracle's result."""
import numpy as np
import pytest
import torch

from paper_2111_09512_amd import workloads as W
from tests.gpu_common import dev, host, need_gpu, say

pytestmark = pytest.mark.gpu

MATS = {
    "poisson9": lambda: W.poisson7(9),
    "vardens9": lambda: W.vardens7(9, seed_rho=4),
    "aniso7": lambda: W.aniso27(7),
    "perm7": lambda: W.permuted_longrange7(7, seed=1),
    "mmatrix2000": lambda: W.random_mmatrix(2000, 0.003, seed=5),
}


@pytest.fixture(scope="module")
def B():
    need_gpu()
    from paper_2111_09512_amd import binding

    return binding


@pytest.fixture(scope="module")
def ctx(B):
    return B.Context()


def _same(gpu, ref):
    np.testing.assert_array_equal(host(gpu.row_ptr), ref.row_ptr)
    np.testing.assert_array_equal(host(gpu.col_idx), ref.col)
    np.testing.assert_array_equal(host(gpu.val), ref.val)


@pytest.mark.parametrize("sweeps", [0, 1, 2, 5, 17])
@pytest.mark.parametrize("name", list(MATS))
def test_sweeps_bitwise(orc, B, ctx, name, sweeps):
    say("fixed point", name, sweeps)
    A = MATS[name]()
    Ls, U, k = orc.ilu0_fixed_point(A, sweeps)
    gL, gU, changed = ctx.ilu0_fixed_point(B.Csr.from_host(A), sweeps)
    _same(gL, Ls)
    _same(gU, U)
    if sweeps > 0:
        assert changed == (k > sweeps - 1)


@pytest.mark.parametrize("name", ["poisson9", "mmatrix2000"])
def test_standstill_is_ilu0_and_drives_the_smoother(orc, B, ctx, name):
    A = MATS[name]()
    Ls0, U0 = orc.ilu0(A)
    _, _, k = orc.ilu0_fixed_point(A, 5000)
    gL, gU, changed = ctx.ilu0_fixed_point(B.Csr.from_host(A), k + 1)
    assert not changed
    _same(gL, Ls0)
    _same(gU, U0)
    d, dinv, Us = orc.scale_rows(U0)
    F = ctx.ilu_scale_factors(gL, gU)
    b = W.rhs(A.n, 0)
    x = dev(np.zeros(A.n))
    ctx.ilu_smooth(B.Csr.from_host(A), F, dev(b), x, 2, 3, 3)
    np.testing.assert_array_equal(host(x), orc.smooth(A, Ls0, Us, dinv, b, np.zeros(A.n), 2, 3, 3))


def test_errors(B, ctx):
    A = W.CSR.from_dense(np.array([[2.0, 0.0], [1.0, 0.0]]))
    A.val[:] = [2.0, 1.0]
    with pytest.raises(B.SiluError) as e:
        ctx.ilu0_fixed_point(B.Csr.from_host(A), 2)
    assert e.value.status == -3 and e.value.row == 1
    with pytest.raises(B.SiluError) as e:
        ctx.ilu0_fixed_point(B.Csr.from_host(W.poisson7(3)), -1)
    assert e.value.status == -1
