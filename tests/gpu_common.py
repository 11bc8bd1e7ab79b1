"""Helpers shared by the GPU parity tests: build the same case for the oracle
(host, FP64) and for the HIP path (device), and compare."""
import numpy as np
import pytest
import torch

F64_TOL = 1e-12  # FP64 path vs the FP64 oracle, relative
MIXED_TOL = 1e-5  # FP32-inner path vs the FP64 oracle, relative


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


def say(*args):
    print("[gpu-test]", *args, flush=True)


class Case:
    """Oracle factors of A (FP64, host) and their device copies, scaled by the library."""

    def __init__(self, orc, B, ctx, A, kind, params, fp32=False, scale=True):
        self.A = A
        self.Ls, self.U = orc.factor(A, kind, params)
        self.d, self.dinv, self.Us = orc.scale_rows(self.U)
        self.Ad = B.Csr.from_host(A)
        self.Ld = B.Csr.from_host(self.Ls)
        self.Ud = B.Csr.from_host(self.U)
        self.F = ctx.ilu_scale_factors(self.Ld, self.Ud, fp32=fp32, scale=scale)
        torch.cuda.synchronize()


def rel_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = max(np.linalg.norm(ref), 1e-300)
    return float(np.linalg.norm(got - ref) / den)


def assert_close(got, ref, tol, what=""):
    """Element by element against tol * ||ref||_inf, and norm-wise against tol."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape
    assert np.all(np.isfinite(got)), f"{what}: non-finite output"
    scale = max(np.abs(ref).max(), 1e-300)
    worst = np.abs(got - ref).max() / scale
    assert worst <= tol, f"{what}: max elementwise error {worst:.3e} > {tol:.1e}"
    assert rel_err(got, ref) <= tol, f"{what}: normwise error {rel_err(got, ref):.3e} > {tol:.1e}"
    return worst


def dev(v):
    return torch.from_numpy(np.ascontiguousarray(v, np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()
