"""ctypes front end of the FP64 CPU oracle (oracle/gsk_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the benchmark's
CPU-baseline leg, never by the product path. All arrays are numpy host arrays.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import numpy as np

from . import build as _build

CONVERGED, MAXIT, BREAKDOWN, STAGNATED = 0, 1, 2, 3
OK, ERR_ARG, ERR_ZERO_ROW, ERR_NONFINITE, ERR_ALLOC = 0, -1, -2, -3, -7
STATUS_NAMES = {CONVERGED: "converged", MAXIT: "maxit", BREAKDOWN: "breakdown",
                STAGNATED: "stagnated"}

_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        lib.orc_gs_scale.restype = ctypes.c_int
        lib.orc_gs_scale.argtypes = [ctypes.c_int, _ip, _ip, _dp, _dp, ctypes.c_int, _dp, _dp,
                                     _dp, _dp]
        lib.orc_spmv.restype = None
        lib.orc_spmv.argtypes = [ctypes.c_int, _ip, _ip, _dp, _dp, _dp]
        lib.orc_ilu0.restype = ctypes.c_int
        lib.orc_ilu0.argtypes = [ctypes.c_int, _ip, _ip, _dp, _dp]
        lib.orc_arnoldi.restype = ctypes.c_int
        lib.orc_arnoldi.argtypes = [ctypes.c_int, _ip, _ip, _dp, _dp, ctypes.c_int, _dp, _dp,
                                    ctypes.c_double]
        lib.orc_gmres.restype = ctypes.c_int
        lib.orc_gmres.argtypes = [ctypes.c_int, _ip, _ip, _dp, _dp, _dp, ctypes.c_int,
                                  ctypes.c_double, ctypes.c_int, ctypes.c_double, _dp, _dp,
                                  _dp, _ip, _dp]
        lib.orc_bicgstab.restype = ctypes.c_int
        lib.orc_bicgstab.argtypes = [ctypes.c_int, _ip, _ip, _dp, _dp, _dp, ctypes.c_double,
                                     ctypes.c_int, ctypes.c_double, _dp, _dp, _dp, _ip, _dp]
        lib.orc_default_breakdown_eps.restype = ctypes.c_double
        lib.orc_gmres_ir.restype = ctypes.c_int
        lib.orc_gmres_ir.argtypes = [ctypes.c_int, _ip, _ip, _dp, _dp, _dp, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_int, ctypes.c_double, _dp, _ip,
                                     _dp]
        lib.orc_bicgstab_ir.restype = ctypes.c_int
        lib.orc_bicgstab_ir.argtypes = [ctypes.c_int, _ip, _ip, _dp, _dp, _dp, ctypes.c_double,
                                        ctypes.c_int, ctypes.c_double, _dp, ctypes.c_double,
                                        ctypes.c_int, ctypes.c_int, _ip, _dp]
        lib.orc_default_breakdown_eps.argtypes = []
        _lib = lib
    return _lib


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _i(a):
    assert a.dtype == np.int32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_ip)


def default_breakdown_eps() -> float:
    return float(_load().orc_default_breakdown_eps())


@dataclasses.dataclass
class Info:
    iters: int
    restarts: int
    status: int
    half_step: int
    verify_failures: int
    relres_recursive: float
    relres_true: float
    breakdown_test: int = 0
    fp64_from: int = 0        # mixed Bi-CGSTAB: iterations before the FP64 continuation (0: none)

    @property
    def status_name(self) -> str:
        return STATUS_NAMES.get(self.status, str(self.status))


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code}")
        self.code = code


def _csr(A):
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(A.col_idx, dtype=np.int32)
    val = np.ascontiguousarray(A.val, dtype=np.float64)
    return rp, ci, val


def gs_scale(A, b, p: int):
    """GS(p) of (A, b). Returns (val_scaled, b_scaled, norms, weights); raises OracleError."""
    rp, ci, val = _csr(A)
    n = rp.shape[0] - 1
    b = np.ascontiguousarray(b, dtype=np.float64)
    vo = np.empty_like(val)
    bo = np.empty_like(b)
    nrm = np.empty(n)
    w = np.empty(n)
    rc = _load().orc_gs_scale(n, _i(rp), _i(ci), _d(val), _d(b), int(p), _d(vo), _d(bo),
                              _d(nrm), _d(w))
    if rc != OK:
        raise OracleError(rc)
    return vo, bo, nrm, w


def spmv(A, x):
    rp, ci, val = _csr(A)
    n = rp.shape[0] - 1
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(n)
    _load().orc_spmv(n, _i(rp), _i(ci), _d(val), _d(x), _d(y))
    return y


def ilu0(A):
    rp, ci, val = _csr(A)
    n = rp.shape[0] - 1
    lu = np.empty_like(val)
    rc = _load().orc_ilu0(n, _i(rp), _i(ci), _d(val), _d(lu))
    if rc != OK:
        raise OracleError(rc)
    return lu


def arnoldi(A, r0, m: int, eps_b: Optional[float] = None):
    """Returns (V [n x (m+1)], H [(m+1) x m], steps) from CGS2 Arnoldi started at r0."""
    rp, ci, val = _csr(A)
    n = rp.shape[0] - 1
    r0 = np.ascontiguousarray(r0, dtype=np.float64)
    V = np.zeros((m + 1, n))      # row l = column l of the basis (column-major storage)
    H = np.zeros((m, m + 1))      # row j = column j of H
    eps = default_breakdown_eps() if eps_b is None else eps_b
    steps = _load().orc_arnoldi(n, _i(rp), _i(ci), _d(val), _d(r0), int(m), _d(V), _d(H), eps)
    if steps < 0:
        raise OracleError(steps)
    return V.T.copy(), H.T.copy(), int(steps)


def _info(ii, dd):
    return Info(int(ii[0]), int(ii[1]), int(ii[2]), int(ii[3]), int(ii[4]), float(dd[0]),
                float(dd[1]), int(ii[5]))


def gmres(A, b, x0=None, m: int = 30, tol: float = 1e-8, maxit: int = 10000,
          eps_b: Optional[float] = None, weights=None, ilu=None, history: bool = False):
    """Restarted GMRES(m) with CGS2 Arnoldi. Returns (x, Info[, hist])."""
    rp, ci, val = _csr(A)
    n = rp.shape[0] - 1
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    hist = np.full(max(maxit, 1), np.nan) if history else None
    ii = np.zeros(6, dtype=np.int32)
    dd = np.zeros(2)
    eps = default_breakdown_eps() if eps_b is None else eps_b
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    lu = None if ilu is None else np.ascontiguousarray(ilu, dtype=np.float64)
    rc = _load().orc_gmres(n, _i(rp), _i(ci), _d(val), _d(b), _d(x), int(m), float(tol),
                           int(maxit), eps, _d(w), _d(lu), _d(hist), _i(ii), _d(dd))
    if rc != OK:
        raise OracleError(rc)
    info = _info(ii, dd)
    if history:
        return x, info, hist[: min(info.iters, maxit)]
    return x, info


def gmres_ir(A, b, x0=None, m: int = 30, tol: float = 1e-8, maxit: int = 10000,
             eps_b: Optional[float] = None, weights=None):
    """Mixed-precision restarted GMRES(m): FP64 residuals and updates, one GMRES(m) cycle with
    float storage per refinement step. Returns (x, Info)."""
    rp, ci, val = _csr(A)
    n = rp.shape[0] - 1
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    ii = np.zeros(6, dtype=np.int32)
    dd = np.zeros(2)
    eps = default_breakdown_eps() if eps_b is None else eps_b
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    rc = _load().orc_gmres_ir(n, _i(rp), _i(ci), _d(val), _d(b), _d(x), int(m), float(tol),
                              int(maxit), eps, _d(w), _i(ii), _d(dd))
    if rc != OK:
        raise OracleError(rc)
    return x, _info(ii, dd)


def bicgstab(A, b, x0=None, tol: float = 1e-8, maxit: int = 10000,
             eps_b: Optional[float] = None, weights=None, ilu=None, history: bool = False):
    """Bi-CGSTAB. Returns (x, Info[, hist])."""
    rp, ci, val = _csr(A)
    n = rp.shape[0] - 1
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    hist = np.full(max(maxit, 1), np.nan) if history else None
    ii = np.zeros(6, dtype=np.int32)
    dd = np.zeros(2)
    eps = default_breakdown_eps() if eps_b is None else eps_b
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    lu = None if ilu is None else np.ascontiguousarray(ilu, dtype=np.float64)
    rc = _load().orc_bicgstab(n, _i(rp), _i(ci), _d(val), _d(b), _d(x), float(tol),
                              int(maxit), eps, _d(w), _d(lu), _d(hist), _i(ii), _d(dd))
    if rc != OK:
        raise OracleError(rc)
    info = _info(ii, dd)
    if history:
        return x, info, hist[: min(info.iters, maxit)]
    return x, info


def bicgstab_ir(A, b, x0=None, tol: float = 1e-8, maxit: int = 10000,
                eps_b: Optional[float] = None, weights=None, delta: float = 2.0 ** -14,
                fallback: bool = True, run_cap: int = 1000):
    """Mixed-precision Bi-CGSTAB: FP64 residuals and x, Bi-CGSTAB runs with float storage
    between them, each ending at a reduction by delta of the residual it started from; with
    fallback, a refinement that stops making progress (or breaks down) continues as FP64
    Bi-CGSTAB; a float run ends after run_cap iterations (0: no cap). Returns (x, Info);
    Info.fp64_from = iterations before the FP64 continuation."""
    rp, ci, val = _csr(A)
    n = rp.shape[0] - 1
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    ii = np.zeros(7, dtype=np.int32)
    dd = np.zeros(2)
    eps = default_breakdown_eps() if eps_b is None else eps_b
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    rc = _load().orc_bicgstab_ir(n, _i(rp), _i(ci), _d(val), _d(b), _d(x), float(tol),
                                 int(maxit), eps, _d(w), float(delta), 1 if fallback else 0,
                                 int(run_cap), _i(ii), _d(dd))
    if rc != OK:
        raise OracleError(rc)
    info = _info(ii, dd)
    info.fp64_from = int(ii[6])
    return x, info
