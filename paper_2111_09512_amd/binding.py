"""Thin Python binding over libscaledilu.so (argument marshalling only).

Every numerical step runs in the library's HIP kernels (or, for the host-side
factorization set-up, in its C++ code); this module only turns torch tensors
into device pointers and sizes, passes the current torch stream, and raises on
a non-zero status.  The entry points keep the C-ABI names: ``ilu_scale_factors``,
``ilu_smooth``, ``trisolve_direct``, ``trisolve_iter``, ``silu_analyze``.

There is no fallback: if the shared library is missing the import fails.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref
from dataclasses import dataclass

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libscaledilu.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
        "(or `python paper_2111_09512_amd/build.py`). There is no CPU fallback."
    )
_lib = C.CDLL(LIB_PATH)

SILU_F64, SILU_F32 = 0, 1
SILU_DIRECT, SILU_MIXED, SILU_CHECK_FINITE, SILU_VALIDATE, SILU_NO_SCALING = 0x1, 0x2, 0x4, 0x8, 0x10
SILU_KERNEL_STREAM, SILU_KERNEL_VECTOR, SILU_KERNEL_BLOCKED = 0x100, 0x200, 0x400
SILU_NO_GRAPH, SILU_INDEX32, SILU_NO_WINDOW, SILU_WINDOW = 0x800, 0x1000, 0x2000, 0x4000
SILU_CODE16, SILU_ZERO_GUESS, SILU_GRAPH, SILU_REORDER = 0x8000, 0x10000, 0x20000, 0x40000
SILU_SLICED_LOOP = 0x80000
SILU_CODE8 = 0x100000
SILU_ROWPAT = 0x400000
SILU_RELABELED = 0x200000
# None: sliced copies (1-byte diagonal codes where they fit, else 2, else 4);
# "sliced16": no diagonal table; "sliced32": 4-byte columns;
# "stream": CSR-stream, 16-bit offsets where they fit, else the LDS window, else col_idx;
# "win": the LDS window wherever it fits; "stream16": offsets at most; "stream32": col_idx always
KERNELS = {None: 0, "rowpat": SILU_ROWPAT, "sliced8": SILU_CODE8, "sliced_loop": SILU_CODE8 | SILU_SLICED_LOOP, "sliced16": SILU_CODE16, "sliced32": SILU_INDEX32, "blocked": SILU_KERNEL_BLOCKED,
           "stream": SILU_KERNEL_STREAM, "vector": SILU_KERNEL_VECTOR, "win": SILU_KERNEL_STREAM | SILU_WINDOW,
           "stream16": SILU_KERNEL_STREAM | SILU_NO_WINDOW, "stream32": SILU_KERNEL_STREAM | SILU_INDEX32}
SILU_LOWER, SILU_UPPER = 0, 1
SILU_UNIT, SILU_NONUNIT = 0, 1

STATUS = {
    0: "SILU_OK", -1: "SILU_ERR_ARG", -2: "SILU_ERR_SHAPE", -3: "SILU_ERR_PATTERN", -4: "SILU_ERR_ZERO_PIVOT",
    -5: "SILU_ERR_NONFINITE", -6: "SILU_ERR_NOMEM", -7: "SILU_ERR_HIP", -8: "SILU_ERR_UNSUPPORTED",
    -9: "SILU_ERR_TIMEOUT",
}


class silu_csr(C.Structure):
    _fields_ = [
        ("n_rows", C.c_int64), ("n_cols", C.c_int64), ("nnz", C.c_int64),
        ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p), ("dtype", C.c_int32),
    ]


class silu_factors(C.Structure):
    _fields_ = [
        ("Ls", silu_csr), ("Us", silu_csr), ("d", C.c_void_p), ("dinv", C.c_void_p),
        ("Ls_val32", C.c_void_p), ("Us_val32", C.c_void_p), ("scaled", C.c_int32), ("dc", C.c_void_p),
    ]


class silu_host_csr(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.POINTER(C.c_int32)),
        ("col_idx", C.POINTER(C.c_int32)), ("val", C.POINTER(C.c_double)),
    ]


_P = C.c_void_p
_sig = {
    "silu_create": (C.c_int, [C.POINTER(_P), _P]),
    "silu_destroy": (C.c_int, [_P]),
    "silu_set_stream": (C.c_int, [_P, _P]),
    "silu_bad_row": (C.c_int64, [_P]),
    "silu_last_hip_error": (C.c_int, [_P]),
    "silu_status_string": (C.c_char_p, [C.c_int]),
    "silu_workspace_size": (C.c_int, [_P, C.c_int64, C.c_int, C.POINTER(C.c_size_t)]),
    "ilu_scale_factors": (C.c_int, [_P, C.POINTER(silu_csr), C.POINTER(silu_csr), C.POINTER(silu_factors), C.c_int]),
    "ilu_scale_factors_rowcol": (C.c_int, [_P, C.POINTER(silu_csr), C.POINTER(silu_csr), C.c_int,
                                           C.POINTER(silu_factors), C.c_int]),
    "gs_split_size": (C.c_int, [_P, C.POINTER(silu_csr), C.POINTER(C.c_int64)]),
    "gs_scale_split": (C.c_int, [_P, C.POINTER(silu_csr), C.POINTER(silu_factors), C.c_int]),
    "gs_smooth": (C.c_int, [_P, C.POINTER(silu_csr), C.POINTER(silu_factors), _P, _P, C.c_int, C.c_int, C.c_int, _P,
                            C.c_size_t]),
    "silu_split_sizes": (C.c_int, [_P, C.POINTER(silu_csr), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "silu_ilu0_fixed_point_workspace_size": (C.c_int, [_P, C.c_int64, C.c_int64, C.POINTER(C.c_size_t)]),
    "silu_ilu0_fixed_point": (C.c_int, [_P, C.POINTER(silu_csr), C.c_int, C.POINTER(silu_csr), C.POINTER(silu_csr),
                                        C.POINTER(C.c_int), C.c_int, _P, C.c_size_t]),
    "silu_fgmres_workspace_size": (C.c_int, [_P, C.c_int64, C.c_int, C.c_int, C.POINTER(C.c_size_t)]),
    "silu_fgmres": (C.c_int, [_P, C.POINTER(silu_csr), C.POINTER(silu_factors), _P, _P, C.c_int, C.c_int,
                              C.c_double, C.c_int, C.c_int, C.c_int, C.c_int, _P, C.c_size_t, C.POINTER(C.c_int),
                              C.POINTER(C.c_double)]),
    "silu_fgmres_nrbe": (C.c_int, [_P, C.POINTER(silu_csr), C.POINTER(silu_factors), _P, _P, C.c_int, C.c_int,
                                   C.c_double, C.c_double, C.c_int, C.c_int, C.c_int, C.c_int, _P, C.c_size_t,
                                   C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "silu_aux_workspace_size": (C.c_int, [C.c_int64, C.POINTER(C.c_size_t)]),
    "silu_norm2_estimate": (C.c_int, [_P, C.POINTER(silu_csr), _P, C.c_int, C.POINTER(C.c_double), _P, C.c_size_t]),
    "silu_nrbe": (C.c_int, [_P, C.POINTER(silu_csr), _P, _P, C.c_double, C.POINTER(C.c_double), _P, C.c_size_t]),
    "silu_spmv": (C.c_int, [_P, C.POINTER(silu_csr), _P, _P, C.c_int]),
    "silu_dot": (C.c_int, [_P, C.c_int64, _P, _P, C.POINTER(C.c_double), _P, C.c_size_t]),
    "ilu_smooth": (C.c_int, [_P, C.POINTER(silu_csr), C.POINTER(silu_factors), _P, _P, C.c_int, C.c_int, C.c_int,
                             _P, C.c_size_t]),
    "ilu_smooth2": (C.c_int, [_P, C.POINTER(silu_csr), C.POINTER(silu_factors), _P, _P, C.c_int, C.c_int,
                              C.c_int, C.c_int, _P, C.c_size_t]),
    "trisolve_direct": (C.c_int, [_P, C.POINTER(silu_csr), C.c_int, C.c_int, _P, _P, C.c_int]),
    "trisolve_iter": (C.c_int, [_P, C.POINTER(silu_csr), _P, _P, _P, C.c_int, C.c_int, _P, C.c_size_t]),
    "silu_analyze": (C.c_int, [_P, C.POINTER(silu_csr), C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "silu_release": (C.c_int, [_P, _P, _P]),
    "silu_set_timing": (C.c_int, [_P, C.c_int]),
    "silu_stats_collect": (C.c_int, [_P]),
    "silu_stats_get": (C.c_int, [_P, C.c_int, C.c_char_p, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                 C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "silu_stats_reset": (C.c_int, [_P]),
    "silu_stream_copy": (C.c_int, [_P, _P, _P, C.c_size_t]),
    "silu_stream_read": (C.c_int, [_P, _P, C.c_size_t, _P]),
    "silu_reorder_vectors": (C.c_int, [_P, _P, _P, _P, _P, C.c_int]),
    "ilu_smooth_noalloc": (C.c_int, [_P, _P, _P, _P, _P, C.c_int, C.c_int, C.c_int, C.c_int]),
    "silu_factor_iluk": (C.c_int, [C.POINTER(silu_host_csr), C.c_int, C.POINTER(silu_host_csr),
                                   C.POINTER(silu_host_csr), C.POINTER(C.c_int64)]),
    "silu_factor_ilut": (C.c_int, [C.POINTER(silu_host_csr), C.c_double, C.c_int, C.POINTER(silu_host_csr),
                                   C.POINTER(silu_host_csr), C.POINTER(C.c_int64)]),
    "silu_host_csr_free": (None, [C.POINTER(silu_host_csr)]),
    "silu_server_create": (C.c_int, [_P, _P, _P, C.c_size_t, C.c_int, C.POINTER(_P)]),
    "silu_server_destroy": (C.c_int, [_P]),
    "silu_server_register": (C.c_int, [_P, C.POINTER(silu_csr), C.POINTER(silu_factors), C.POINTER(C.c_int)]),
    "silu_server_request_bytes": (C.c_int64, [_P, C.c_int]),
    "silu_server_submit": (C.c_int, [_P, C.c_int, _P, _P, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int64)]),
    "silu_server_submit_flags": (C.c_int, [_P, C.c_int, _P, _P, C.c_int, C.c_int, C.c_int, C.c_int,
                                           C.POINTER(C.c_int64)]),
    "silu_server_submit_solve": (C.c_int, [_P, C.c_int, _P, _P, C.c_double, C.c_int, C.c_int, C.c_int,
                                           C.POINTER(C.c_int64)]),
    "silu_server_solve_result": (C.c_int, [_P, C.c_int64, C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "silu_server_step": (C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "silu_server_poll": (C.c_int, [_P, C.c_int64, C.POINTER(C.c_int)]),
    "silu_server_last_hip_error": (C.c_int, [_P]),
    "silu_server_set_mode": (C.c_int, [_P, C.c_int, C.c_int]),
    "silu_server_completed": (C.c_int, [_P, C.POINTER(C.c_int64), C.c_int, C.POINTER(C.c_int)]),
    "silu_server_run": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "silu_server_wait": (C.c_int, [_P, C.c_int64]),
    "silu_server_times": (C.c_int, [_P, C.c_int64, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "silu_server_footprint": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "silu_reorder_rcm": (C.c_int, [C.c_int64, _P, _P, _P, C.c_double, _P]),
    "silu_server_set_wait_limit": (C.c_int, [_P, C.c_int]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


class SiluError(RuntimeError):
    def __init__(self, status: int, where: str, row: int = -1, hip: int = 0):
        msg = f"{where}: {STATUS.get(status, status)} ({_lib.silu_status_string(status).decode()})"
        if row >= 0:
            msg += f", row {row}"
        if hip:
            msg += f", hip error {hip}"
        super().__init__(msg)
        self.status = status
        self.row = row


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


# --------------------------------------------------------------------------
# device containers
# --------------------------------------------------------------------------

@dataclass
class Csr:
    """Device CSR: int32 row_ptr / col_idx, float64 (or float32) values, torch tensors."""

    row_ptr: torch.Tensor
    col_idx: torch.Tensor
    val: torch.Tensor

    @property
    def n(self) -> int:
        return self.row_ptr.numel() - 1

    @property
    def nnz(self) -> int:
        return self.col_idx.numel()

    def c(self) -> silu_csr:
        for t in (self.row_ptr, self.col_idx, self.val):
            if not t.is_contiguous():
                raise ValueError("CSR arrays must be contiguous")
        if self.row_ptr.dtype != torch.int32 or self.col_idx.dtype != torch.int32:
            raise TypeError("row_ptr and col_idx must be int32")
        dt = {torch.float64: SILU_F64, torch.float32: SILU_F32}[self.val.dtype]
        return silu_csr(self.n, self.n, self.nnz, self.row_ptr.data_ptr(), _ptr(self.col_idx) if self.nnz else None,
                        _ptr(self.val) if self.nnz else None, dt)

    @staticmethod
    def from_host(M, device="cuda") -> "Csr":
        """Upload a host CSR (anything with row_ptr, col, val numpy arrays)."""
        return Csr(torch.from_numpy(np.ascontiguousarray(M.row_ptr, np.int32)).to(device),
                   torch.from_numpy(np.ascontiguousarray(M.col, np.int32)).to(device),
                   torch.from_numpy(np.ascontiguousarray(M.val, np.float64)).to(device))


@dataclass
class Factors:
    Ls: Csr
    Us: Csr
    d: torch.Tensor
    dinv: torch.Tensor
    Ls_val32: torch.Tensor | None
    Us_val32: torch.Tensor | None
    scaled: int  # 0 unscaled, 1 row scaling, 2 row/column scaling
    dc: torch.Tensor | None = None  # column factors (scaled == 2)

    def c(self) -> silu_factors:
        return silu_factors(self.Ls.c(), self.Us.c(), _ptr(self.d), _ptr(self.dinv), _ptr(self.Ls_val32),
                            _ptr(self.Us_val32), int(self.scaled), _ptr(self.dc))

    def nbytes(self) -> int:
        ts = [self.Ls.row_ptr, self.Ls.col_idx, self.Ls.val, self.Us.row_ptr, self.Us.col_idx, self.Us.val, self.d,
              self.dinv, self.Ls_val32, self.Us_val32, self.dc]
        return sum(t.numel() * t.element_size() for t in ts if t is not None)


# --------------------------------------------------------------------------
# context
# --------------------------------------------------------------------------

class Context:
    """Owns a silu_ctx bound to a torch stream (default: the current stream)."""

    def __init__(self, stream: torch.cuda.Stream | None = None):
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        st = _lib.silu_create(C.byref(h), C.c_void_p(self.stream.cuda_stream))
        if st:
            raise SiluError(st, "silu_create")
        self._h = h
        self._ws = None
        self._tracked = set()
        self._versions = {}

    def _track(self, *mats, values=()):
        """The library caches analyses and sliced copies of a matrix keyed by
        its pointers: release them when its arrays are freed, and when a value
        array (the matrix's own, or an extra one such as an FP32 copy) has been
        changed in place since the last call (torch's version counter)."""
        for k, M in enumerate(mats):
            key = (M.row_ptr.data_ptr(), M.col_idx.data_ptr() if M.nnz else 0)
            vals = [M.val] + [v for v in (values[k] if k < len(values) else ()) if v is not None]
            vers = tuple((v.data_ptr(), v._version) for v in vals)
            if key in self._tracked:
                seen = dict(self._versions.get(key, ()))
                if any(seen.get(ptr, ver) != ver for ptr, ver in vers):  # changed in place
                    _lib.silu_release(self._h, C.c_void_p(key[0]), C.c_void_p(key[1] or None))
                self._versions[key] = vers
                continue
            self._tracked.add(key)
            self._versions[key] = vers
            ref = weakref.ref(self)
            weakref.finalize(M.row_ptr, _release_cb, ref, key)
            for v in vals:
                weakref.finalize(v, _release_cb, ref, key)

    def close(self):
        if getattr(self, "_h", None):
            _lib.silu_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, where: str):
        if st:
            raise SiluError(st, where, int(_lib.silu_bad_row(self._h)), int(_lib.silu_last_hip_error(self._h)))

    # ---- workspace ----
    def workspace_size(self, n: int, flags: int = 0) -> int:
        b = C.c_size_t()
        self._check(_lib.silu_workspace_size(self._h, n, flags, C.byref(b)), "silu_workspace_size")
        return b.value

    def workspace(self, n: int, flags: int = 0) -> torch.Tensor:
        need = self.workspace_size(n, flags)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        return self._ws

    # ---- setup ----
    @staticmethod
    def _alloc_factors(L: Csr, U: Csr, fp32: bool, scaled: int) -> tuple[Factors, silu_factors]:
        n = U.n
        nnz_s = U.nnz - n
        dev = U.val.device
        Us = Csr(torch.empty(n + 1, dtype=torch.int32, device=dev), torch.empty(max(nnz_s, 0), dtype=torch.int32,
                                                                               device=dev),
                 torch.empty(max(nnz_s, 0), dtype=torch.float64, device=dev))
        F = Factors(L, Us, torch.empty(n, dtype=torch.float64, device=dev),
                    torch.empty(n, dtype=torch.float64, device=dev),
                    torch.empty(L.nnz, dtype=torch.float32, device=dev) if fp32 else None,
                    torch.empty(max(nnz_s, 0), dtype=torch.float32, device=dev) if fp32 else None, scaled,
                    torch.empty(n, dtype=torch.float64, device=dev) if scaled == 2 else None)
        Fc = F.c()
        Fc.Us = silu_csr(n, n, max(nnz_s, 0), Us.row_ptr.data_ptr(), _ptr(Us.col_idx) if nnz_s else None,
                         _ptr(Us.val) if nnz_s else None, SILU_F64)
        return F, Fc

    def ilu_scale_factors(self, L: Csr, U: Csr, fp32: bool = False, scale: bool = True,
                          validate: bool = False) -> Factors:
        F, Fc = self._alloc_factors(L, U, fp32, 1 if scale else 0)
        flags = (0 if scale else SILU_NO_SCALING) | (SILU_VALIDATE if validate else 0)
        Lc, Uc = L.c(), U.c()
        self._check(_lib.ilu_scale_factors(self._h, C.byref(Lc), C.byref(Uc), C.byref(Fc), flags), "ilu_scale_factors")
        return F

    def ilu_scale_factors_rowcol(self, L: Csr, U: Csr, ruiz_iters: int = 5, fp32: bool = False,
                                 validate: bool = False) -> Factors:
        """Row/column scaling U^ = D_r U D_c with a unit diagonal (F.dinv = d_r, F.dc = d_c)."""
        F, Fc = self._alloc_factors(L, U, fp32, 2)
        Lc, Uc = L.c(), U.c()
        self._check(_lib.ilu_scale_factors_rowcol(self._h, C.byref(Lc), C.byref(Uc), int(ruiz_iters), C.byref(Fc),
                                                  SILU_VALIDATE if validate else 0), "ilu_scale_factors_rowcol")
        return F

    # ---- ILU(0) on the device by fixed-point sweeps ----
    def ilu0_fixed_point(self, A: Csr, sweeps: int, validate: bool = False):
        """Returns (Ls, U, changed): ILU(0) after `sweeps` synchronous fixed-point sweeps."""
        Ac = A.c()
        nl, nu = C.c_int64(), C.c_int64()
        self._check(_lib.silu_split_sizes(self._h, C.byref(Ac), C.byref(nl), C.byref(nu)), "silu_split_sizes")
        dev = A.val.device
        Ls = Csr(torch.empty(A.n + 1, dtype=torch.int32, device=dev), torch.empty(nl.value, dtype=torch.int32, device=dev),
                 torch.empty(nl.value, dtype=torch.float64, device=dev))
        U = Csr(torch.empty(A.n + 1, dtype=torch.int32, device=dev), torch.empty(nu.value, dtype=torch.int32, device=dev),
                torch.empty(nu.value, dtype=torch.float64, device=dev))
        nb = C.c_size_t()
        self._check(_lib.silu_ilu0_fixed_point_workspace_size(self._h, A.n, A.nnz, C.byref(nb)),
                    "silu_ilu0_fixed_point_workspace_size")
        ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
        Lc, Uc = Ls.c(), U.c()
        ch = C.c_int()
        self._check(_lib.silu_ilu0_fixed_point(self._h, C.byref(Ac), int(sweeps), C.byref(Lc), C.byref(Uc),
                                               C.byref(ch), SILU_VALIDATE if validate else 0,
                                               C.c_void_p(ws.data_ptr()), ws.numel()), "silu_ilu0_fixed_point")
        return Ls, U, bool(ch.value)

    # ---- Krylov solver around the smoother ----
    def fgmres(self, A: Csr, F: Factors, b: torch.Tensor, x: torch.Tensor, restart: int = 30, max_iters: int = 300,
               tol: float = 1e-8, outer: int = 1, m_L: int = 3, m_U: int = 3, mixed: bool = False,
               kernel: str | None = None, check_finite: bool = False, reorder: bool = False,
               norm_a: float | None = None):
        """FGMRES(restart) with the smoother as right preconditioner, in place on x.
        Stops on the relative residual (eq. relres), or, given norm_a = ||A||_2 (or
        its estimate), on the norm-wise relative backward error (eq. nbre).
        Returns (steps, history of the estimates)."""
        _vec(b, A.n, "b")
        _vec(x, A.n, "x")
        flags = ((SILU_MIXED if mixed else 0) | (SILU_CHECK_FINITE if check_finite else 0) |
                 (SILU_REORDER if reorder else 0) | KERNELS[kernel])
        nb = C.c_size_t()
        self._check(_lib.silu_fgmres_workspace_size(self._h, A.n, restart, flags, C.byref(nb)),
                    "silu_fgmres_workspace_size")
        if getattr(self, "_kws", None) is None or self._kws.numel() < nb.value:
            self._kws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        hist = np.zeros(max_iters + 1)
        it = C.c_int()
        self._track(A, F.Ls, F.Us, values=((), (F.Ls_val32,), (F.Us_val32,)))
        Ac, Fc = A.c(), F.c()
        tail = (outer, m_L, m_U, flags, C.c_void_p(self._kws.data_ptr()), self._kws.numel(), C.byref(it),
                hist.ctypes.data_as(C.POINTER(C.c_double)))
        if norm_a is None:
            self._check(_lib.silu_fgmres(self._h, C.byref(Ac), C.byref(Fc), C.c_void_p(b.data_ptr()),
                                         C.c_void_p(x.data_ptr()), restart, max_iters, tol, *tail), "silu_fgmres")
        else:
            self._check(_lib.silu_fgmres_nrbe(self._h, C.byref(Ac), C.byref(Fc), C.c_void_p(b.data_ptr()),
                                              C.c_void_p(x.data_ptr()), restart, max_iters, tol, float(norm_a),
                                              *tail), "silu_fgmres_nrbe")
        return it.value, hist[: it.value + 1].copy()

    def spmv(self, A: Csr, xin: torch.Tensor, y: torch.Tensor | None = None, kernel: str | None = None):
        """y = A x."""
        _vec(xin, A.n, "x")
        y = torch.empty_like(xin) if y is None else y
        self._track(A)
        Ac = A.c()
        self._check(_lib.silu_spmv(self._h, C.byref(Ac), C.c_void_p(xin.data_ptr()), C.c_void_p(y.data_ptr()),
                                   KERNELS[kernel]), "silu_spmv")
        return y

    def dot(self, a: torch.Tensor, b: torch.Tensor) -> float:
        if getattr(self, "_dws", None) is None:
            self._dws = torch.empty(8448, dtype=torch.uint8, device="cuda")
        out = C.c_double()
        self._check(_lib.silu_dot(self._h, a.numel(), C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()),
                                  C.byref(out), C.c_void_p(self._dws.data_ptr()), self._dws.numel()), "silu_dot")
        return out.value

    def _aux_ws(self, n: int) -> torch.Tensor:
        nb = C.c_size_t()
        self._check(_lib.silu_aux_workspace_size(n, C.byref(nb)), "silu_aux_workspace_size")
        if getattr(self, "_aws", None) is None or self._aws.numel() < nb.value:
            self._aws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        return self._aws

    def norm2_estimate(self, A: Csr, iters: int = 30, seed: int = 0) -> float:
        """Power-iteration estimate of ||A||_2 (exact in the limit for a symmetric
        A, a lower bound otherwise), for the NRBE of eq. nbre; the random start
        vector is drawn here from `seed`."""
        g = torch.Generator(device="cpu").manual_seed(seed)
        v0 = (torch.rand(A.n, generator=g, dtype=torch.float64) - 0.5).cuda()
        ws = self._aux_ws(A.n)
        self._track(A)
        Ac, out = A.c(), C.c_double()
        self._check(_lib.silu_norm2_estimate(self._h, C.byref(Ac), C.c_void_p(v0.data_ptr()), iters, C.byref(out),
                                             C.c_void_p(ws.data_ptr()), ws.numel()), "silu_norm2_estimate")
        return out.value

    def nrbe(self, A: Csr, b: torch.Tensor, x: torch.Tensor, norm_a: float) -> float:
        """Norm-wise relative backward error ||b - A x|| / (||b|| + ||A|| ||x||) (eq. nbre)."""
        _vec(b, A.n, "b")
        _vec(x, A.n, "x")
        ws = self._aux_ws(A.n)
        self._track(A)
        Ac, out = A.c(), C.c_double()
        self._check(_lib.silu_nrbe(self._h, C.byref(Ac), C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                                   float(norm_a), C.byref(out), C.c_void_p(ws.data_ptr()), ws.numel()), "silu_nrbe")
        return out.value

    # ---- polynomial Gauss-Seidel ----
    def gs_split(self, A: Csr, fp32: bool = False, validate: bool = False) -> Factors:
        """Gs = D^{-1} L (strictly lower part of A, row-scaled), d, dinv for gs_smooth."""
        Ac = A.c()
        cnt = C.c_int64()
        self._check(_lib.gs_split_size(self._h, C.byref(Ac), C.byref(cnt)), "gs_split_size")
        n, nnz, dev = A.n, cnt.value, A.val.device
        Gs = Csr(torch.empty(n + 1, dtype=torch.int32, device=dev), torch.empty(nnz, dtype=torch.int32, device=dev),
                 torch.empty(nnz, dtype=torch.float64, device=dev))
        empty = Csr(torch.zeros(n + 1, dtype=torch.int32, device=dev), torch.empty(0, dtype=torch.int32, device=dev),
                    torch.empty(0, dtype=torch.float64, device=dev))
        G = Factors(Gs, empty, torch.empty(n, dtype=torch.float64, device=dev),
                    torch.empty(n, dtype=torch.float64, device=dev),
                    torch.empty(nnz, dtype=torch.float32, device=dev) if fp32 else None, None, 3)
        Gc = G.c()
        self._check(_lib.gs_scale_split(self._h, C.byref(Ac), C.byref(Gc), SILU_VALIDATE if validate else 0),
                    "gs_scale_split")
        return G

    def gs_smooth(self, A: Csr, G: Factors, b: torch.Tensor, x: torch.Tensor, outer_sweeps: int, terms: int,
                  mixed: bool = False, check_finite: bool = False, validate: bool = False, kernel: str | None = None,
                  ws: torch.Tensor | None = None, reorder: bool = False) -> torch.Tensor:
        """x <- x + sum_{j<terms} (-D^{-1}L)^j D^{-1}(b - A x), `outer_sweeps` times, in place."""
        flags = ((SILU_MIXED if mixed else 0) | (SILU_CHECK_FINITE if check_finite else 0) |
                 (SILU_VALIDATE if validate else 0) | (SILU_REORDER if reorder else 0) | KERNELS[kernel])
        _vec(b, A.n, "b")
        _vec(x, A.n, "x")
        ws = self.workspace(A.n, flags) if ws is None else ws
        self._track(A, G.Ls, values=((), (G.Ls_val32,)))
        Ac, Gc = A.c(), G.c()
        self._check(_lib.gs_smooth(self._h, C.byref(Ac), C.byref(Gc), C.c_void_p(b.data_ptr()),
                                   C.c_void_p(x.data_ptr()), outer_sweeps, terms, flags, C.c_void_p(ws.data_ptr()),
                                   ws.numel()), "gs_smooth")
        return x

    # ---- the smoother ----
    def ilu_smooth(self, A: Csr, F: Factors, b: torch.Tensor, x: torch.Tensor, outer_sweeps: int, m_L: int,
                   m_U: int | None = None, direct: bool = False, mixed: bool = False, check_finite: bool = False,
                   validate: bool = False, kernel: str | None = None, ws: torch.Tensor | None = None,
                   graph: bool = True, zero_guess: bool = False, record: bool = False,
                   reorder: bool = False, relabeled: bool = False) -> torch.Tensor:
        """x <- x + M^{-1}(b - A x), `outer_sweeps` times, in place on x (returned).
        zero_guess: x holds zeros on entry (the first residual is b).
        record: replay the call's sweep sequence from a hipGraph recorded on the
        first call with the same tensors and counts (SILU_GRAPH).
        reorder: sweep locality-relabeled copies (SILU_REORDER; same results).
        relabeled: with reorder, b and x are already in the copies' order (reorder_vectors)."""
        m_U = m_L if m_U is None else m_U
        flags = ((SILU_DIRECT if direct else 0) | (SILU_MIXED if mixed else 0) | (SILU_ZERO_GUESS if zero_guess else 0) |
                 (SILU_CHECK_FINITE if check_finite else 0) | (SILU_VALIDATE if validate else 0) |
                 (0 if graph else SILU_NO_GRAPH) | (SILU_GRAPH if record else 0) |
                 (SILU_REORDER if reorder else 0) | (SILU_RELABELED if relabeled else 0) | KERNELS[kernel])
        _vec(b, A.n, "b")
        _vec(x, A.n, "x")
        ws = self.workspace(A.n, flags) if ws is None else ws
        self._track(A, F.Ls, F.Us, values=((), (F.Ls_val32,), (F.Us_val32,)))
        Ac, Fc = A.c(), F.c()
        self._check(_lib.ilu_smooth2(self._h, C.byref(Ac), C.byref(Fc), C.c_void_p(b.data_ptr()),
                                     C.c_void_p(x.data_ptr()), outer_sweeps, m_L, m_U, flags,
                                     C.c_void_p(ws.data_ptr()), ws.numel()), "ilu_smooth")
        return x

    def ilu_smooth_noalloc(self, A: Csr, F: Factors, b: torch.Tensor, x: torch.Tensor, outer_sweeps: int, m_L: int,
                           m_U: int | None = None, mixed: bool = False, zero_guess: bool = False,
                           check_finite: bool = False, kernel: str | None = None) -> torch.Tensor:
        """ilu_smooth with its work vectors in the library's per-device scratch array
        (no workspace, no allocation), in place on x."""
        m_U = m_L if m_U is None else m_U
        flags = ((SILU_MIXED if mixed else 0) | (SILU_ZERO_GUESS if zero_guess else 0) |
                 (SILU_CHECK_FINITE if check_finite else 0) | KERNELS[kernel])
        _vec(b, A.n, "b")
        _vec(x, A.n, "x")
        self._track(A, F.Ls, F.Us, values=((), (F.Ls_val32,), (F.Us_val32,)))
        Ac, Fc = A.c(), F.c()
        self._check(_lib.ilu_smooth_noalloc(self._h, C.byref(Ac), C.byref(Fc), C.c_void_p(b.data_ptr()),
                                            C.c_void_p(x.data_ptr()), outer_sweeps, m_L, m_U, flags),
                    "ilu_smooth_noalloc")
        return x

    def reorder_vectors(self, A: Csr, F: Factors, src: torch.Tensor, to_relabeled: bool = True,
                        out: torch.Tensor | None = None) -> torch.Tensor:
        """src moved into the order of the SILU_REORDER copies of (A, F), or back."""
        _vec(src, A.n, "src")
        out = torch.empty_like(src) if out is None else out
        self._track(A, F.Ls, F.Us, values=((), (F.Ls_val32,), (F.Us_val32,)))
        Ac, Fc = A.c(), F.c()
        self._check(_lib.silu_reorder_vectors(self._h, C.byref(Ac), C.byref(Fc), C.c_void_p(src.data_ptr()),
                                              C.c_void_p(out.data_ptr()), 1 if to_relabeled else 0),
                    "silu_reorder_vectors")
        return out

    def trisolve_direct(self, T: Csr, uplo: int, diag: int, rhs: torch.Tensor, out: torch.Tensor | None = None,
                        validate: bool = False, graph: bool = True) -> torch.Tensor:
        _vec(rhs, T.n, "rhs")
        out = torch.empty_like(rhs) if out is None else out
        self._track(T)
        Tc = T.c()
        self._check(_lib.trisolve_direct(self._h, C.byref(Tc), uplo, diag, C.c_void_p(rhs.data_ptr()),
                                         C.c_void_p(out.data_ptr()),
                                         (SILU_VALIDATE if validate else 0) | (0 if graph else SILU_NO_GRAPH)),
                    "trisolve_direct")
        return out

    def trisolve_iter(self, T: Csr, rhs: torch.Tensor, m: int, dinv: torch.Tensor | None = None,
                      out: torch.Tensor | None = None, kernel: str | None = None) -> torch.Tensor:
        _vec(rhs, T.n, "rhs")
        out = torch.empty_like(rhs) if out is None else out
        flags = KERNELS[kernel]
        ws = self.workspace(T.n, 0)
        self._track(T)
        Tc = T.c()
        self._check(_lib.trisolve_iter(self._h, C.byref(Tc), C.c_void_p(_ptr(dinv)), C.c_void_p(rhs.data_ptr()),
                                       C.c_void_p(out.data_ptr()), m, flags, C.c_void_p(ws.data_ptr()),
                                       ws.numel()), "trisolve_iter")
        return out

    def silu_analyze(self, T: Csr, uplo: int):
        depth = C.c_int32()
        self._track(T)
        Tc = T.c()
        self._check(_lib.silu_analyze(self._h, C.byref(Tc), uplo, C.byref(depth), None), "silu_analyze")
        rows = (C.c_int32 * max(depth.value, 1))()
        self._check(_lib.silu_analyze(self._h, C.byref(Tc), uplo, C.byref(depth), rows), "silu_analyze")
        return depth.value, np.ctypeslib.as_array(rows)[: depth.value].copy()

    # ---- measurement ----
    def set_timing(self, on: bool):
        self._check(_lib.silu_set_timing(self._h, 1 if on else 0), "silu_set_timing")

    def stats(self) -> dict:
        k = _lib.silu_stats_collect(self._h)
        if k < 0:
            self._check(k, "silu_stats_collect")
        out = {}
        buf = C.create_string_buffer(64)
        for i in range(k):
            la, ms, by, lb = C.c_int64(), C.c_double(), C.c_double(), C.c_double()
            self._check(_lib.silu_stats_get(self._h, i, buf, 64, C.byref(la), C.byref(ms), C.byref(by), C.byref(lb)),
                        "silu_stats_get")
            out[buf.value.decode()] = {"launches": la.value, "ms": ms.value, "bytes": by.value,
                                       "layout_bytes": lb.value}
        return out

    def stats_reset(self):
        self._check(_lib.silu_stats_reset(self._h), "silu_stats_reset")

    def stream_copy(self, src: torch.Tensor, dst: torch.Tensor):
        nb = src.numel() * src.element_size()
        self._check(_lib.silu_stream_copy(self._h, C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nb),
                    "silu_stream_copy")

    def stream_read(self, src: torch.Tensor, out: torch.Tensor):
        """Read-dominant calibration stream: reads all of src (a multiple of 49,152 bytes),
        writes src's bytes / 24 to out."""
        nb = src.numel() * src.element_size()
        if out.numel() * out.element_size() < nb // 24:
            raise ValueError("stream_read: out holds fewer than bytes / 24 bytes")
        self._check(_lib.silu_stream_read(self._h, C.c_void_p(src.data_ptr()), nb, C.c_void_p(out.data_ptr())),
                    "silu_stream_read")


def _release_cb(ctx_ref, key):
    ctx = ctx_ref()
    if ctx is not None and getattr(ctx, "_h", None) and key in ctx._tracked:
        _lib.silu_release(ctx._h, C.c_void_p(key[0]), C.c_void_p(key[1] or None))
        ctx._tracked.discard(key)
        ctx._versions.pop(key, None)


def _vec(t: torch.Tensor, n: int, what: str):
    if t.dtype != torch.float64 or t.numel() != n or not t.is_contiguous() or not t.is_cuda:
        raise ValueError(f"{what} must be a contiguous float64 CUDA tensor of length {n}")


# --------------------------------------------------------------------------
# host-side factorization set-up (silu_factor.h)
# --------------------------------------------------------------------------

@dataclass
class HostCsr:
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


def _host_in(A) -> tuple[silu_host_csr, tuple]:
    rp = np.ascontiguousarray(A.row_ptr, np.int32)
    col = np.ascontiguousarray(A.col, np.int32)
    val = np.ascontiguousarray(A.val, np.float64)
    h = silu_host_csr(int(A.n), int(rp[-1]), rp.ctypes.data_as(C.POINTER(C.c_int32)),
                      col.ctypes.data_as(C.POINTER(C.c_int32)), val.ctypes.data_as(C.POINTER(C.c_double)))
    return h, (rp, col, val)


def _host_out(h: silu_host_csr) -> HostCsr:
    n, nnz = int(h.n), int(h.nnz)
    rp = np.ctypeslib.as_array(h.row_ptr, shape=(n + 1,)).copy()
    if nnz:
        col = np.ctypeslib.as_array(h.col_idx, shape=(nnz,)).copy()
        val = np.ctypeslib.as_array(h.val, shape=(nnz,)).copy()
    else:
        col, val = np.zeros(0, np.int32), np.zeros(0)
    _lib.silu_host_csr_free(C.byref(h))
    return HostCsr(n, rp, col, val)


def factor_iluk(A, k: int) -> tuple[HostCsr, HostCsr]:
    """ILU(k) on the host (set-up): returns (strictly lower L, upper U with diagonal first)."""
    h, keep = _host_in(A)
    L, U, bad = silu_host_csr(), silu_host_csr(), C.c_int64(-1)
    st = _lib.silu_factor_iluk(C.byref(h), int(k), C.byref(L), C.byref(U), C.byref(bad))
    if st:
        raise SiluError(st, f"silu_factor_iluk(k={k})", int(bad.value))
    return _host_out(L), _host_out(U)


def factor_ilut(A, tau: float, p: int) -> tuple[HostCsr, HostCsr]:
    """ILUT(tau, p) on the host (set-up)."""
    h, keep = _host_in(A)
    L, U, bad = silu_host_csr(), silu_host_csr(), C.c_int64(-1)
    st = _lib.silu_factor_ilut(C.byref(h), float(tau), int(p), C.byref(L), C.byref(U), C.byref(bad))
    if st:
        raise SiluError(st, f"silu_factor_ilut(tau={tau}, p={p})", int(bad.value))
    return _host_out(L), _host_out(U)


def reorder_rcm(A, theta: float = 0.25) -> np.ndarray:
    """The SILU_REORDER relabeling of a host CSR matrix: order[k] = the row
    placed at position k (reverse Cuthill-McKee on the strong couplings)."""
    rp = np.ascontiguousarray(A.row_ptr, np.int32)
    col = np.ascontiguousarray(A.col, np.int32)
    val = np.ascontiguousarray(A.val, np.float64)
    order = np.empty(A.n, np.int32)
    st = _lib.silu_reorder_rcm(int(A.n), rp.ctypes.data, col.ctypes.data, val.ctypes.data, float(theta),
                               order.ctypes.data)
    if st:
        raise SiluError(st, "silu_reorder_rcm")
    return order


def factor(A, kind: str, params: dict) -> tuple[HostCsr, HostCsr]:
    if kind == "ilu0":
        return factor_iluk(A, 0)
    if kind == "iluk":
        return factor_iluk(A, params["k"])
    if kind == "ilut":
        return factor_ilut(A, params["tau"], params["p"])
    raise KeyError(kind)


# --------------------------------------------------------------------------
# serving (continuous batching on resident matrices)
# --------------------------------------------------------------------------

class Server:
    """Wraps a silu_server.  The arena (device workspace budget) is a torch
    tensor owned here; registered matrices and request vectors are kept
    referenced until the server is closed, so the device pointers stay valid."""

    QUEUED, RUNNING, LAUNCHED, DONE = 0, 1, 2, 3
    STEPWISE, PERSISTENT = 0, 1

    def __init__(self, ctx: Context, arena_bytes: int, max_active: int = 256, persistent: bool = False,
                 max_workgroups: int = 0):
        self.ctx = ctx
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
        h = C.c_void_p()
        st = _lib.silu_server_create(ctx._h, C.c_void_p(ctx.stream.cuda_stream), C.c_void_p(self.arena.data_ptr()),
                                     arena_bytes, max_active, C.byref(h))
        if st:
            raise SiluError(st, "silu_server_create")
        self._h = h
        self._keep = []
        self._req = {}
        if persistent:
            self.set_mode(self.PERSISTENT, max_workgroups)

    def set_mode(self, mode: int, max_workgroups: int = 0):
        """STEPWISE (one batched launch per sweep) or PERSISTENT (one launch
        per admitted batch running every sweep of its requests)."""
        self._check(_lib.silu_server_set_mode(self._h, mode, max_workgroups), "silu_server_set_mode")

    def set_wait_limit(self, microseconds: int):
        """Wall-clock bound of one wait inside a persistent launch, in microseconds (0: default)."""
        self._check(_lib.silu_server_set_wait_limit(self._h, microseconds), "silu_server_set_wait_limit")

    def close(self):
        if getattr(self, "_h", None):
            _lib.silu_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, where):
        if st:
            raise SiluError(st, where, hip=int(_lib.silu_server_last_hip_error(self._h)))

    def register(self, A: Csr, F: Factors) -> int:
        mid = C.c_int()
        Ac, Fc = A.c(), F.c()
        self._check(_lib.silu_server_register(self._h, C.byref(Ac), C.byref(Fc), C.byref(mid)), "silu_server_register")
        self._keep.append((A, F))
        return mid.value

    def request_bytes(self, mid: int) -> int:
        return int(_lib.silu_server_request_bytes(self._h, mid))

    def submit(self, mid: int, b: torch.Tensor, x: torch.Tensor, outer: int, m_L: int, m_U: int,
               mixed: bool = False) -> int:
        """A smoother request; mixed: the FP32-inner form (factors with FP32 values)."""
        t = C.c_int64()
        if mixed:
            self._check(_lib.silu_server_submit_flags(self._h, mid, C.c_void_p(b.data_ptr()),
                                                      C.c_void_p(x.data_ptr()), outer, m_L, m_U, SILU_MIXED,
                                                      C.byref(t)), "silu_server_submit_flags")
        else:
            self._check(_lib.silu_server_submit(self._h, mid, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                                                outer, m_L, m_U, C.byref(t)), "silu_server_submit")
        self._req[t.value] = (b, x)
        return t.value

    def submit_solve(self, mid: int, b: torch.Tensor, x: torch.Tensor, tol: float, max_outer: int, m_L: int,
                     m_U: int) -> int:
        """A solve request: outer steps until ||b - A x|| / ||b|| < tol (checked for x0 and
        after each step), at most max_outer."""
        t = C.c_int64()
        self._check(_lib.silu_server_submit_solve(self._h, mid, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                                                  float(tol), max_outer, m_L, m_U, C.byref(t)),
                    "silu_server_submit_solve")
        self._req[t.value] = (b, x)
        return t.value

    def solve_result(self, ticket: int) -> tuple[int, float]:
        """(outer steps after which the test passed, or max_outer + 1; relative residual of
        the last check) of a finished solve request."""
        k, rel = C.c_int(), C.c_double()
        self._check(_lib.silu_server_solve_result(self._h, ticket, C.byref(k), C.byref(rel)),
                    "silu_server_solve_result")
        return k.value, rel.value

    def step(self) -> tuple[int, int]:
        a, q = C.c_int(), C.c_int()
        self._check(_lib.silu_server_step(self._h, C.byref(a), C.byref(q)), "silu_server_step")
        return a.value, q.value

    def run(self, max_steps: int) -> tuple[int, int]:
        """Up to max_steps scheduling steps in one call."""
        a, q = C.c_int(), C.c_int()
        self._check(_lib.silu_server_run(self._h, max_steps, C.byref(a), C.byref(q)), "silu_server_run")
        return a.value, q.value

    def completed(self, capacity: int = 1024) -> list:
        """Tickets of the requests found done since the last call (each once)."""
        buf = getattr(self, "_done_buf", None)
        if buf is None or len(buf) < capacity:
            buf = self._done_buf = (C.c_int64 * capacity)()
        k = C.c_int()
        self._check(_lib.silu_server_completed(self._h, buf, capacity, C.byref(k)), "silu_server_completed")
        out = [int(buf[i]) for i in range(k.value)]
        for t in out:
            self._req.pop(t, None)
        return out

    def wait(self, ticket: int):
        """Block until the request is done (steps the server as needed)."""
        self._check(_lib.silu_server_wait(self._h, ticket), "silu_server_wait")
        self._req.pop(ticket, None)

    def times(self, ticket: int) -> tuple[float, float | None]:
        """(submitted, found done) on the host's steady clock, in seconds."""
        a, d = C.c_int64(), C.c_int64()
        self._check(_lib.silu_server_times(self._h, ticket, C.byref(a), C.byref(d)), "silu_server_times")
        return a.value * 1e-9, (d.value * 1e-9 if d.value >= 0 else None)

    def footprint(self) -> tuple[int, int, int]:
        """(ticket records, pinned result slots, done tickets not yet returned by completed)."""
        r, p, u = C.c_int64(), C.c_int64(), C.c_int64()
        self._check(_lib.silu_server_footprint(self._h, C.byref(r), C.byref(p), C.byref(u)), "silu_server_footprint")
        return r.value, p.value, u.value

    def poll(self, ticket: int) -> int:
        st = C.c_int()
        self._check(_lib.silu_server_poll(self._h, ticket, C.byref(st)), "silu_server_poll")
        if st.value == self.DONE:
            self._req.pop(ticket, None)
        return st.value
