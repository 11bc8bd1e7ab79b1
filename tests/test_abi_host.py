"""CPU tests of libscaledilu.so: it loads, exports every function its headers
declare, rejects bad arguments on the host, and its host-side factorization
set-up agrees with the oracle's factorization (no GPU needed for any of it)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2111_09512_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2111_09512_amd", "libscaledilu.so")


def header_functions():
    names = set()
    for h in ("scaled_ilu.h", "silu_factor.h"):
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", src, re.M):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libscaledilu.so is not built (run __graft_entry__.build())")
    return C.CDLL(LIB)


def test_library_exports_every_declared_function(lib):
    names = header_functions()
    assert {"ilu_scale_factors", "ilu_smooth", "ilu_smooth2", "trisolve_direct", "trisolve_iter", "silu_create",
            "silu_workspace_size", "silu_factor_iluk", "silu_factor_ilut"} <= names
    for nm in sorted(names):
        assert hasattr(lib, nm), nm


def test_binding_declares_the_same_names():
    from paper_2111_09512_amd import binding as B

    assert set(B.EXPORTED) == header_functions()


def test_host_side_argument_errors(lib):
    lib.silu_status_string.restype = C.c_char_p
    assert lib.silu_status_string(0) == b"ok"
    assert lib.silu_status_string(-4) == b"zero or non-finite pivot"
    lib.silu_workspace_size.argtypes = [C.c_void_p, C.c_int64, C.c_int, C.c_void_p]
    assert lib.silu_workspace_size(None, 10, 0, None) == -1
    lib.ilu_smooth2.argtypes = [C.c_void_p] * 5 + [C.c_int] * 4 + [C.c_void_p, C.c_size_t]
    assert lib.ilu_smooth2(None, None, None, None, None, 1, 1, 1, 0, None, 0) == -1
    lib.silu_create.argtypes = [C.c_void_p, C.c_void_p]
    assert lib.silu_create(None, None) == -1


def _same(a, b):
    assert a.n == b.n
    np.testing.assert_array_equal(a.row_ptr, b.row_ptr)
    np.testing.assert_array_equal(a.col, b.col)
    np.testing.assert_array_equal(a.val, b.val)


@pytest.mark.parametrize("make,kind,params", [
    (lambda: W.poisson7(10), "ilu0", {}),
    (lambda: W.vardens7(9), "iluk", {"k": 1}),
    (lambda: W.vardens7(7), "iluk", {"k": 2}),
    (lambda: W.random_mmatrix(80, 0.08, 3), "iluk", {"k": 3}),
    (lambda: W.aniso27(9), "ilut", {"tau": 1e-3, "p": 20}),
    (lambda: W.random_mmatrix(70, 0.2, 4), "ilut", {"tau": 0.02, "p": 4}),
    (lambda: W.permuted_longrange7(8), "ilu0", {}),
])
def test_host_factorization_matches_oracle_bitwise(orc, make, kind, params):
    """The library's set-up factorization and the oracle's are independent
    implementations of the same definitions with the same operation order, so
    the factors agree bit for bit (patterns and values)."""
    from paper_2111_09512_amd import binding as B

    A = make()
    L, U = B.factor(A, kind, params)
    Lo, Uo = orc.factor(A, kind, params)
    _same(L, Lo)
    _same(U, Uo)


def test_host_factorization_errors():
    from paper_2111_09512_amd import binding as B

    M = np.array([[2.0, 1.0, 0.0], [1.0, 0.0, 1.0], [0.0, 1.0, 2.0]])
    A = W.CSR.from_dense(M)  # row 1 stores no diagonal
    with pytest.raises(B.SiluError) as e:
        B.factor_iluk(A, 0)
    assert e.value.status == -3 and e.value.row == 1
    Z = W.CSR.from_dense(np.array([[1.0, 1.0], [1.0, 1.0]]))  # u_11 = 0 after elimination
    with pytest.raises(B.SiluError) as e:
        B.factor_iluk(Z, 0)
    assert e.value.status == -4 and e.value.row == 1
    with pytest.raises(B.SiluError) as e:
        B.factor_ilut(Z, 0.0, 5)
    assert e.value.status == -4
