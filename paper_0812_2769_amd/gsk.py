"""ctypes binding of libgsk.so (include/gsk.h): argument marshalling only.

Torch CUDA tensors supply device memory and the stream; every computation runs in the HIP
library. Importing this module loads the library and raises ImportError if it has not been
built (python -m paper_0812_2769_amd.build); there is no fallback path.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional, Tuple

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgsk.so")

# Return codes and outcomes (include/gsk.h)
OK = 0
ERR_INVALID_ARG, ERR_ZERO_ROW, ERR_NONFINITE, ERR_WORKSPACE, ERR_DEVICE = -1, -2, -3, -4, -5
CONVERGED, MAXIT, BREAKDOWN, STAGNATED = 0, 1, 2, 3
STATUS_NAMES = {CONVERGED: "converged", MAXIT: "maxit", BREAKDOWN: "breakdown",
                STAGNATED: "stagnated"}
METHOD_GS, METHOD_GMRES, METHOD_BICGSTAB, METHOD_ARNOLDI, METHOD_GMRES_MIXED = 0, 1, 2, 3, 4
MAX_RESTART = 64
BRK_NONE, BRK_SIGMA, BRK_OMEGA, BRK_RHO, BRK_GIVENS = 0, 1, 2, 3, 4


class GskError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gsk error {code}: {msg}")
        self.code = code


class Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class Stencil(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("coef", ctypes.c_void_p)]


class Matrix(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("csr", Csr), ("stencil", Stencil)]


MATRIX_CSR, MATRIX_STENCIL = 0, 1


class Options(ctypes.Structure):
    _fields_ = [("maxit", ctypes.c_int32), ("breakdown_eps", ctypes.c_double),
                ("stop_weights", ctypes.c_void_p), ("check_every", ctypes.c_int32)]


class InfoStruct(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("status", ctypes.c_int32), ("half_step", ctypes.c_int32),
                ("verify_failures", ctypes.c_int32), ("breakdown_test", ctypes.c_int32),
                ("fp64_from", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("relres_recursive", ctypes.c_double),
                ("relres_true", ctypes.c_double)]


class ProbeResult(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("busy_launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_int64), ("info", InfoStruct)]


class EngineUsage(ctypes.Structure):
    _fields_ = [("active", ctypes.c_int32), ("max_systems", ctypes.c_int32),
                ("max_rows", ctypes.c_int64), ("free_rows", ctypes.c_int64),
                ("largest_free_rows", ctypes.c_int64)]


ENGINE_GRAPH = 1
FULL = 1
PRECISION_FP64, PRECISION_MIXED = 0, 1


class EngineConfig(ctypes.Structure):
    _fields_ = [("max_rows", ctypes.c_int64), ("max_systems", ctypes.c_int32),
                ("method", ctypes.c_int32), ("m", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("tile_units", ctypes.c_int32), ("inner_reduction", ctypes.c_double),
                ("run_cap", ctypes.c_int32), ("class_shapes", ctypes.c_int32)]


# Size classes of an FP64 Bi-CGSTAB engine with per-class launch shapes (gsk_engine_config):
# 2D stencils and CSR, 3D stencils under 2^18 rows, larger 3D stencils; and the shape codes.
SIZE_CLASSES = ("2d", "3d_small", "3d_large")
CLASS_LARGE_ROWS = 1 << 18
SHAPE_TILE, SHAPE_PAIR_TILE_U, SHAPE_PAIR = 1, 2, 3
SHAPES = {"tile": SHAPE_TILE, "pair_tile_u": SHAPE_PAIR_TILE_U, "pair": SHAPE_PAIR}


def size_class(A) -> str:
    """The size class of a matrix in an engine with per-class shapes."""
    if isinstance(A, StencilMatrix) and A.nz > 1:
        return "3d_large" if A.n >= CLASS_LARGE_ROWS else "3d_small"
    return "2d"


def encode_class_shapes(shapes) -> int:
    """{class name: shape name or code} -> gsk_engine_config.class_shapes."""
    code = 0
    for c, v in (shapes or {}).items():
        k = SIZE_CLASSES.index(c)
        code |= (SHAPES[v] if isinstance(v, str) else int(v)) << (4 * k)
    return code


class EngineRequest(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("b", ctypes.c_void_p), ("x", ctypes.c_void_p),
                ("tol", ctypes.c_double), ("opt", ctypes.c_void_p), ("tag", ctypes.c_int64),
                ("gs_p", ctypes.c_int32), ("val_out", ctypes.c_void_p),
                ("b_out", ctypes.c_void_p), ("stop_weight_out", ctypes.c_void_p),
                ("mat32", ctypes.c_void_p), ("mat32_ld", ctypes.c_int64)]

KCLASS = {"gmres_a": 1, "gmres_b": 2, "gmres_c": 3, "bicg_p": 4, "bicg_s": 5, "bicg_u": 6,
          "residual": 7, "gmres_x": 8, "batch_p": 9, "batch_s": 10, "batch_u": 11}
SOLVER_KCLASSES = ("gmres_a", "gmres_b", "gmres_c", "bicg_p", "bicg_s", "bicg_u", "residual",
                   "gmres_x")
ENGINE_KCLASSES = ("batch_p", "batch_s", "batch_u")


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_0812_2769_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    lib.gsk_default_options.argtypes = [P(Options)]
    lib.gsk_default_options.restype = None
    lib.gsk_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.gsk_workspace_bytes.restype = sz
    lib.gsk_workspace_bytes_for.argtypes = [P(Matrix), ctypes.c_int32, ctypes.c_int32]
    lib.gsk_workspace_bytes_for.restype = sz
    lib.gsk_gs_scale.argtypes = [P(Csr), vp, ctypes.c_int32, vp, vp, vp, vp, vp, sz, vp]
    lib.gsk_gs_scale.restype = ctypes.c_int
    lib.gsk_spmv.argtypes = [P(Matrix), vp, vp, vp]
    lib.gsk_spmv.restype = ctypes.c_int
    lib.gsk_stencil_from_csr.argtypes = [P(Csr), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         vp, vp, sz, vp]
    lib.gsk_stencil_from_csr.restype = ctypes.c_int
    lib.gsk_arnoldi.argtypes = [P(Matrix), vp, ctypes.c_int32, vp, ctypes.c_int64, vp,
                                P(ctypes.c_int32), vp, sz, vp]
    lib.gsk_arnoldi.restype = ctypes.c_int
    lib.gsk_gmres.argtypes = [P(Matrix), vp, vp, ctypes.c_int32, ctypes.c_double, P(Options),
                              P(InfoStruct), vp, sz, vp]
    lib.gsk_gmres.restype = ctypes.c_int
    lib.gsk_gmres_mixed.argtypes = [P(Matrix), vp, vp, ctypes.c_int32, ctypes.c_double,
                                    P(Options), P(InfoStruct), vp, sz, vp]
    lib.gsk_gmres_mixed.restype = ctypes.c_int
    lib.gsk_bicgstab.argtypes = [P(Matrix), vp, vp, ctypes.c_double, P(Options), P(InfoStruct),
                                 vp, sz, vp]
    lib.gsk_bicgstab.restype = ctypes.c_int
    lib.gsk_bicgstab_noalloc.argtypes = [P(Matrix), vp, vp, ctypes.c_double, P(Options),
                                         P(InfoStruct), vp]
    lib.gsk_bicgstab_noalloc.restype = ctypes.c_int
    lib.gsk_bicgstab_noalloc_max_bytes.argtypes = []
    lib.gsk_bicgstab_noalloc_max_bytes.restype = sz
    lib.gsk_probe_begin.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.gsk_probe_begin.restype = ctypes.c_int
    lib.gsk_probe_end.argtypes = [P(ProbeResult)]
    lib.gsk_stream_mix_bytes.restype = sz
    lib.gsk_stream_mix_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64]
    lib.gsk_stream_mix_ms.restype = ctypes.c_int
    lib.gsk_stream_mix_ms.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, vp, sz,
                                      ctypes.c_int32, P(ctypes.c_float), vp]
    lib.gsk_probe_end.restype = ctypes.c_int
    lib.gsk_last_error.argtypes = []
    lib.gsk_last_error.restype = ctypes.c_char_p
    lib.gsk_version.argtypes = []
    lib.gsk_version.restype = ctypes.c_int
    lib.gsk_engine_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int32]
    lib.gsk_engine_workspace_bytes.restype = sz
    lib.gsk_engine_create.argtypes = [vp, sz, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32, vp, P(vp)]
    lib.gsk_engine_create.restype = ctypes.c_int
    lib.gsk_engine_submit.argtypes = [vp, P(Matrix), vp, vp, ctypes.c_double, P(Options),
                                      ctypes.c_int64]
    lib.gsk_engine_submit.restype = ctypes.c_int
    lib.gsk_engine_submit_gs.argtypes = [vp, P(Matrix), vp, ctypes.c_int32, vp, vp, vp, vp,
                                         ctypes.c_double, P(Options), ctypes.c_int64]
    lib.gsk_engine_submit_gs.restype = ctypes.c_int
    lib.gsk_engine_workspace_bytes_ex.argtypes = [P(EngineConfig)]
    lib.gsk_engine_workspace_bytes_ex.restype = sz
    lib.gsk_engine_create_ex.argtypes = [P(EngineConfig), vp, sz, vp, P(vp)]
    lib.gsk_engine_create_ex.restype = ctypes.c_int
    lib.gsk_engine_submit_ex.argtypes = [vp, P(EngineRequest)]
    lib.gsk_engine_submit_ex.restype = ctypes.c_int
    lib.gsk_engine_run.argtypes = [vp, ctypes.c_int32]
    lib.gsk_engine_run.restype = ctypes.c_int
    lib.gsk_engine_poll.argtypes = [vp, ctypes.c_int32, P(Result), ctypes.c_int32,
                                    P(ctypes.c_int32)]
    lib.gsk_engine_poll.restype = ctypes.c_int
    lib.gsk_engine_get_usage.argtypes = [vp, P(EngineUsage)]
    lib.gsk_engine_get_usage.restype = ctypes.c_int
    lib.gsk_engine_destroy.argtypes = [vp]
    lib.gsk_engine_destroy.restype = ctypes.c_int
    lib.gsk_bicgstab_batch_workspace_bytes.argtypes = [ctypes.c_int32, P(ctypes.c_int32)]
    lib.gsk_bicgstab_batch_workspace_bytes.restype = sz
    lib.gsk_bicgstab_batch.argtypes = [ctypes.c_int32, P(Matrix), P(vp), P(vp), ctypes.c_double,
                                       P(Options), P(InfoStruct), vp, sz, vp]
    lib.gsk_bicgstab_batch.restype = ctypes.c_int
    return lib


lib = _load()


def _check(rc: int) -> None:
    if rc != OK:
        raise GskError(rc, lib.gsk_last_error().decode())


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _vec(t: torch.Tensor, n: int, name: str) -> torch.Tensor:
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be a contiguous CUDA float64 tensor of {n} elements")
    return t


def _opt_vec(t: Optional[torch.Tensor], n: int, name: str) -> Optional[int]:
    """Device pointer of an optional float64 vector of n elements (None stays None)."""
    return None if t is None else _vec(t, n, name).data_ptr()


def _ws(ws: torch.Tensor):
    """(pointer, bytes) of a workspace tensor: contiguous device memory of any element type."""
    if not ws.is_cuda or not ws.is_contiguous():
        raise ValueError("ws must be a contiguous CUDA tensor")
    return ws.data_ptr(), ws.numel() * ws.element_size()


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
    fp64_from: int = 0   # mixed Bi-CGSTAB engine: iterations before the FP64 continuation

    @property
    def status_name(self) -> str:
        return STATUS_NAMES.get(self.status, str(self.status))


class CsrMatrix:
    """A CSR matrix in device memory: int32 row_ptr/col_idx, float64 val (torch tensors)."""

    def __init__(self, row_ptr: torch.Tensor, col_idx: torch.Tensor, val: torch.Tensor):
        for name, t, dt in (("row_ptr", row_ptr, torch.int32), ("col_idx", col_idx, torch.int32),
                            ("val", val, torch.float64)):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous CUDA {dt} tensor")
        if col_idx.numel() != val.numel():
            raise ValueError("col_idx and val differ in length")
        self.row_ptr, self.col_idx, self.val = row_ptr, col_idx, val
        self.n = row_ptr.numel() - 1
        self.nnz = val.numel()
        self.device = val.device

    @classmethod
    def from_numpy(cls, row_ptr, col_idx, val, device="cuda") -> "CsrMatrix":
        return cls(torch.as_tensor(row_ptr, dtype=torch.int32).to(device).contiguous(),
                   torch.as_tensor(col_idx, dtype=torch.int32).to(device).contiguous(),
                   torch.as_tensor(val, dtype=torch.float64).to(device).contiguous())

    @classmethod
    def from_problem(cls, problem, device="cuda") -> "CsrMatrix":
        return cls.from_numpy(problem.row_ptr, problem.col_idx, problem.val, device)

    def with_values(self, val: torch.Tensor) -> "CsrMatrix":
        return CsrMatrix(self.row_ptr, self.col_idx, val)

    def c_struct(self) -> Csr:
        return Csr(self.n, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr(),
                   self.val.data_ptr())

    def c_matrix(self) -> Matrix:
        return Matrix(MATRIX_CSR, self.c_struct(), Stencil(0, 0, 0, None))


class StencilMatrix:
    """A structured 5/7-point stencil matrix in device memory (gsk_stencil): an nx x ny x nz
    grid (nz = 1 for 2D) and coefficient planes coef[planes, n] in the CSR column order
    -z, -y, -x, centre, +x, +y, +z."""

    def __init__(self, nx: int, ny: int, nz: int, coef: torch.Tensor):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.n = self.nx * self.ny * self.nz
        planes = 7 if self.nz > 1 else 5
        if (coef.dtype != torch.float64 or not coef.is_cuda or not coef.is_contiguous()
                or coef.numel() != planes * self.n):
            raise ValueError(f"coef must be a contiguous CUDA float64 tensor of {planes}*n values")
        self.coef = coef
        self.device = coef.device

    @property
    def planes(self) -> int:
        return 7 if self.nz > 1 else 5

    def c_matrix(self) -> Matrix:
        return Matrix(MATRIX_STENCIL, Csr(0, 0, None, None, None),
                      Stencil(self.nx, self.ny, self.nz, self.coef.data_ptr()))


def workspace_bytes(method: int, n: int, m: int = 0) -> int:
    return int(lib.gsk_workspace_bytes(method, n, m))


def workspace_bytes_for(A, method: int, m: int = 0) -> int:
    """Exact workspace bytes of `method` for the matrix A (CsrMatrix or StencilMatrix)."""
    c = A.c_matrix()
    return int(lib.gsk_workspace_bytes_for(ctypes.byref(c), method, m))


def _aligned(nbytes: int, device) -> torch.Tensor:
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + nbytes]


def workspace(method: int, n: int, m: int = 0, device="cuda") -> torch.Tensor:
    nbytes = workspace_bytes(method, n, m)
    if nbytes == 0:
        raise GskError(ERR_INVALID_ARG, f"no workspace size for method={method} n={n} m={m}")
    return _aligned(nbytes, device)


def workspace_for(A, method: int, m: int = 0) -> torch.Tensor:
    """A 256-byte aligned workspace of workspace_bytes_for(A, method, m) bytes."""
    nbytes = workspace_bytes_for(A, method, m)
    if nbytes == 0:
        raise GskError(ERR_INVALID_ARG, lib.gsk_last_error().decode() or
                       f"no workspace size for method={method} m={m}")
    return _aligned(nbytes, A.device)


def default_options() -> Options:
    o = Options()
    lib.gsk_default_options(ctypes.byref(o))
    return o


def gs_scale(A: CsrMatrix, b: torch.Tensor, p: int = 2, *, inplace: bool = False,
             want_norms: bool = True, want_weights: bool = False,
             ws: Optional[torch.Tensor] = None):
    """GS(p): returns (A_scaled, b_scaled, row_norms or None, stop_weights or None)."""
    _vec(b, A.n, "b")
    val_out = A.val if inplace else torch.empty_like(A.val)
    b_out = b if inplace else torch.empty_like(b)
    norms = torch.empty(A.n, dtype=torch.float64, device=A.device) if want_norms else None
    weights = torch.empty(A.n, dtype=torch.float64, device=A.device) if want_weights else None
    if ws is None:
        ws = workspace(METHOD_GS, A.n, 0, A.device)
    c = A.c_struct()
    _check(lib.gsk_gs_scale(ctypes.byref(c), b.data_ptr(), int(p), val_out.data_ptr(),
                            b_out.data_ptr(), _ptr(norms), _ptr(weights), *_ws(ws),
                            _stream(A.device)))
    return A.with_values(val_out), b_out, norms, weights


def gs_scale_into(A: CsrMatrix, b: torch.Tensor, p: int, val_out: torch.Tensor,
                  b_out: torch.Tensor, weights: Optional[torch.Tensor] = None, *,
                  norms: Optional[torch.Tensor] = None,
                  ws: Optional[torch.Tensor] = None) -> None:
    """GS(p) into caller-provided outputs (gsk_gs_scale): scaled values, b, and optionally
    stop weights and row norms."""
    _vec(b, A.n, "b")
    _vec(b_out, A.n, "b_out")
    if (val_out.numel() != A.val.numel() or val_out.dtype != torch.float64
            or not val_out.is_cuda or not val_out.is_contiguous()):
        raise GskError(ERR_INVALID_ARG, "val_out must be a contiguous CUDA tensor of nnz "
                                        "float64 values")
    if ws is None:
        ws = workspace(METHOD_GS, A.n, 0, A.device)
    c = A.c_struct()
    _check(lib.gsk_gs_scale(ctypes.byref(c), b.data_ptr(), int(p), val_out.data_ptr(),
                            b_out.data_ptr(), _opt_vec(norms, A.n, "norms"),
                            _opt_vec(weights, A.n, "weights"), *_ws(ws),
                            _stream(A.device)))


def spmv(A, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """y = A x for a CsrMatrix or StencilMatrix."""
    _vec(x, A.n, "x")
    y = torch.empty_like(x) if out is None else _vec(out, A.n, "out")
    c = A.c_matrix()
    _check(lib.gsk_spmv(ctypes.byref(c), x.data_ptr(), y.data_ptr(), _stream(A.device)))
    return y


def stencil_from_csr(A: CsrMatrix, nx: int, ny: int, nz: int = 1,
                     out: Optional[torch.Tensor] = None,
                     ws: Optional[torch.Tensor] = None) -> StencilMatrix:
    """Pack a CSR matrix with a 5/7-point pattern into a StencilMatrix."""
    planes = 7 if nz > 1 else 5
    coef = (torch.empty(planes * A.n, dtype=torch.float64, device=A.device) if out is None
            else _vec(out, planes * A.n, "out"))
    if ws is None:
        ws = workspace(METHOD_GS, A.n, 0, A.device)
    c = A.c_struct()
    _check(lib.gsk_stencil_from_csr(ctypes.byref(c), int(nx), int(ny), int(nz), coef.data_ptr(),
                                    *_ws(ws), _stream(A.device)))
    return StencilMatrix(nx, ny, nz, coef)


def arnoldi(A, r0: torch.Tensor, m: int, ws: Optional[torch.Tensor] = None):
    """CGS2 Arnoldi: returns (V [n x (m+1)] column-major storage as a (m+1, n) tensor
    transposed view, H [(m+1) x m], steps)."""
    _vec(r0, A.n, "r0")
    Vs = torch.zeros((m + 1, A.n), dtype=torch.float64, device=A.device)
    Hs = torch.zeros((m, m + 1), dtype=torch.float64, device=A.device)
    steps = ctypes.c_int32(0)
    if ws is None:
        ws = workspace(METHOD_ARNOLDI, A.n, m, A.device)
    c = A.c_matrix()
    _check(lib.gsk_arnoldi(ctypes.byref(c), r0.data_ptr(), int(m), Vs.data_ptr(), A.n,
                           Hs.data_ptr(), ctypes.byref(steps), *_ws(ws),
                           _stream(A.device)))
    return Vs.t(), Hs.t(), int(steps.value)


def _options(maxit, breakdown_eps, stop_weights, check_every, n) -> Options:
    o = default_options()
    if maxit is not None:
        o.maxit = int(maxit)
    if breakdown_eps is not None:
        o.breakdown_eps = float(breakdown_eps)
    if stop_weights is not None:
        o.stop_weights = _vec(stop_weights, n, "stop_weights").data_ptr()
    if check_every is not None:
        o.check_every = int(check_every)
    return o


def _info(s: InfoStruct) -> Info:
    return Info(s.iters, s.restarts, s.status, s.half_step, s.verify_failures,
                s.relres_recursive, s.relres_true, s.breakdown_test, s.fp64_from)


def _x_start(b, x0, x_out, n):
    if x_out is not None:
        x = _vec(x_out, n, "x_out")
        if x0 is None:
            x.zero_()
        elif x0.data_ptr() != x.data_ptr():
            x.copy_(x0)
        return x
    return torch.zeros_like(b) if x0 is None else _vec(x0, n, "x0").clone()


def gmres(A, b: torch.Tensor, x0: Optional[torch.Tensor] = None, m: int = 30,
          tol: float = 1e-8, *, maxit: Optional[int] = None, breakdown_eps=None,
          stop_weights: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
          x_out: Optional[torch.Tensor] = None):
    """Restarted GMRES(m) with CGS2 Arnoldi. Returns (x, Info)."""
    _vec(b, A.n, "b")
    x = _x_start(b, x0, x_out, A.n)
    if ws is None:
        ws = workspace(METHOD_GMRES, A.n, m, A.device)
    o = _options(maxit, breakdown_eps, stop_weights, None, A.n)
    info = InfoStruct()
    c = A.c_matrix()
    _check(lib.gsk_gmres(ctypes.byref(c), b.data_ptr(), x.data_ptr(), int(m), float(tol),
                         ctypes.byref(o), ctypes.byref(info), *_ws(ws),
                         _stream(A.device)))
    return x, _info(info)


def gmres_mixed(A, b: torch.Tensor, x0: Optional[torch.Tensor] = None, m: int = 30,
                tol: float = 1e-8, *, maxit: Optional[int] = None, breakdown_eps=None,
                stop_weights: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
                x_out: Optional[torch.Tensor] = None):
    """GMRES(m) with FP32 Arnoldi cycles and FP64 restarts (iterative refinement). x, b and
    the matrix stay FP64; the FP32 copies live in the workspace. Returns (x, Info)."""
    _vec(b, A.n, "b")
    x = _x_start(b, x0, x_out, A.n)
    if ws is None:
        ws = workspace_for(A, METHOD_GMRES_MIXED, m)
    o = _options(maxit, breakdown_eps, stop_weights, None, A.n)
    info = InfoStruct()
    c = A.c_matrix()
    _check(lib.gsk_gmres_mixed(ctypes.byref(c), b.data_ptr(), x.data_ptr(), int(m), float(tol),
                               ctypes.byref(o), ctypes.byref(info), *_ws(ws),
                               _stream(A.device)))
    return x, _info(info)


def bicgstab(A, b: torch.Tensor, x0: Optional[torch.Tensor] = None,
             tol: float = 1e-8, *, maxit: Optional[int] = None, breakdown_eps=None,
             stop_weights: Optional[torch.Tensor] = None, check_every: Optional[int] = None,
             ws: Optional[torch.Tensor] = None, x_out: Optional[torch.Tensor] = None):
    """Bi-CGSTAB. Returns (x, Info)."""
    _vec(b, A.n, "b")
    x = _x_start(b, x0, x_out, A.n)
    if ws is None:
        ws = workspace(METHOD_BICGSTAB, A.n, 0, A.device)
    o = _options(maxit, breakdown_eps, stop_weights, check_every, A.n)
    info = InfoStruct()
    c = A.c_matrix()
    _check(lib.gsk_bicgstab(ctypes.byref(c), b.data_ptr(), x.data_ptr(), float(tol),
                            ctypes.byref(o), ctypes.byref(info), *_ws(ws),
                            _stream(A.device)))
    return x, _info(info)


def bicgstab_noalloc(A, b: torch.Tensor, x: torch.Tensor, tol: float = 1e-8, *,
                     maxit: Optional[int] = None, breakdown_eps=None,
                     stop_weights: Optional[torch.Tensor] = None,
                     check_every: Optional[int] = None) -> Info:
    """Bi-CGSTAB through gsk_bicgstab_noalloc: no workspace argument (the library's fixed
    scratch array); x holds x0 on entry and the solution on return. Returns Info."""
    _vec(b, A.n, "b")
    _vec(x, A.n, "x")
    o = _options(maxit, breakdown_eps, stop_weights, check_every, A.n)
    info = InfoStruct()
    c = A.c_matrix()
    _check(lib.gsk_bicgstab_noalloc(ctypes.byref(c), b.data_ptr(), x.data_ptr(), float(tol),
                                    ctypes.byref(o), ctypes.byref(info), _stream(A.device)))
    return _info(info)


def bicgstab_noalloc_max_bytes() -> int:
    return int(lib.gsk_bicgstab_noalloc_max_bytes())


def probe_begin(kernel_class: str, sample_every: int = 1) -> None:
    """Start timing every sample_every-th launch of one kernel class (gsk_probe_begin)."""
    _check(lib.gsk_probe_begin(KCLASS[kernel_class], int(sample_every)))


def probe_end() -> dict:
    r = ProbeResult()
    _check(lib.gsk_probe_end(ctypes.byref(r)))
    return {"launches": r.launches, "busy_launches": r.busy_launches, "total_ms": r.total_ms,
            "bytes": r.bytes}


def stream_mix(reads: int, writes: int, n: int, reps: int = 10, device="cuda") -> dict:
    """The memory ceiling of a streaming mix (gsk_stream_mix_ms): `reads` arrays read and
    `writes` written, n doubles each, best of `reps` launches. Returns the time, the bytes per
    launch and the rate."""
    nbytes = int(lib.gsk_stream_mix_bytes(int(reads), int(writes), int(n)))
    if nbytes == 0:
        raise GskError(ERR_INVALID_ARG, f"unsupported stream mix ({reads}, {writes}) or n")
    dev = torch.device(device)
    buf = torch.zeros(nbytes // 8, dtype=torch.float64, device=dev)
    ms = ctypes.c_float(0.0)
    _check(lib.gsk_stream_mix_ms(int(reads), int(writes), int(n), buf.data_ptr(), nbytes,
                                 int(reps), ctypes.byref(ms), _stream(dev)))
    moved = 8 * (reads + writes) * n
    return {"reads": reads, "writes": writes, "n": n, "best_ms": ms.value,
            "bytes": moved, "GBs": moved / (ms.value * 1e-3) / 1e9}


def _vec_ld(n: int) -> int:
    return (n + 63) // 64 * 64


class Engine:
    """The batch engine with continuous admission (gsk_engine_*): Bi-CGSTAB or GMRES(m), in FP64
    or mixed precision (FP32 storage, FP64 refinement). Systems are submitted with device
    tensors that must stay alive until the system is reported by poll(); results are
    (tag, Info) pairs. The engine's vectors live in a workspace tensor it owns."""

    def __init__(self, max_rows: int, max_systems: int, check_every: int = 8,
                 graph: bool = False, device="cuda", stream=None, method: str = "bicgstab",
                 m: int = 20, precision: str = "fp64", inner_reduction: float = 0.0,
                 tile_units: int = 0, run_cap: int = 0, class_shapes=None):
        self.device = torch.device(device)
        self.stream = stream if stream is not None else (
            torch.cuda.Stream(self.device) if graph else torch.cuda.current_stream(self.device))
        if method not in ("bicgstab", "gmres") or precision not in ("fp64", "mixed"):
            raise ValueError("method must be 'bicgstab' or 'gmres', precision 'fp64' or 'mixed'")
        self.method, self.m = method, int(m)
        self.mixed = precision == "mixed"
        cfg = EngineConfig(int(max_rows), int(max_systems),
                           METHOD_GMRES if method == "gmres" else METHOD_BICGSTAB,
                           self.m if method == "gmres" else 0,
                           PRECISION_MIXED if self.mixed else PRECISION_FP64,
                           int(check_every), ENGINE_GRAPH if graph else 0, int(tile_units),
                           float(inner_reduction), int(run_cap),
                           encode_class_shapes(class_shapes))
        nbytes = int(lib.gsk_engine_workspace_bytes_ex(ctypes.byref(cfg)))
        if nbytes == 0:
            raise GskError(ERR_INVALID_ARG, "no engine workspace size for this configuration")
        self.ws = _aligned(nbytes, self.device)
        h = ctypes.c_void_p()
        _check(lib.gsk_engine_create_ex(ctypes.byref(cfg), self.ws.data_ptr(), self.ws.numel(),
                                        self.stream.cuda_stream, ctypes.byref(h)))
        self._h = h
        self._keep = {}
        self.max_systems = int(max_systems)

    def request_bytes(self, A, p: int = 2) -> int:
        """Device bytes submit_gs allocates for a request on A (scaled matrix, b and, for
        p != 2, stop weights; the FP32 matrix copy in a mixed engine), not counting x."""
        vals = A.coef.numel() if isinstance(A, StencilMatrix) else A.val.numel()
        nbytes = 8 * (vals + A.n + (A.n if p != 2 else 0))
        if self.mixed:
            nbytes += 4 * (A.planes * _vec_ld(A.n) if isinstance(A, StencilMatrix) else vals)
        return nbytes

    @staticmethod
    def workspace_bytes_per_row(method: str = "bicgstab", precision: str = "fp64",
                                m: int = 20) -> float:
        """Engine workspace bytes per row of capacity (measured on a 2^20-row engine with
        256 slots)."""
        rows = 1 << 20
        cfg = EngineConfig(rows, 256, METHOD_GMRES if method == "gmres" else METHOD_BICGSTAB,
                           m if method == "gmres" else 0,
                           PRECISION_MIXED if precision == "mixed" else PRECISION_FP64, 8, 0, 0,
                           0.0, 0, 0)
        return int(lib.gsk_engine_workspace_bytes_ex(ctypes.byref(cfg))) / rows

    def _mat32(self, A) -> Tuple[Optional[torch.Tensor], int]:
        if not self.mixed:
            return None, 0
        if isinstance(A, StencilMatrix):
            ld = _vec_ld(A.n)
            return torch.empty(A.planes * ld, dtype=torch.float32, device=self.device), ld
        return torch.empty(A.nnz, dtype=torch.float32, device=self.device), 0

    def _submit(self, A, b, x, tol, tag, o, gs_p=0, val_out=None, b_out=None, w_out=None,
                keep=()):
        if int(tag) in self._keep:
            raise GskError(ERR_INVALID_ARG, f"tag {int(tag)} is already in flight")
        c = A.c_matrix()
        m32, ld = self._mat32(A)
        r = EngineRequest(ctypes.addressof(c), b.data_ptr(), x.data_ptr(), float(tol),
                          ctypes.addressof(o), int(tag), int(gs_p), _ptr(val_out), _ptr(b_out),
                          _ptr(w_out), _ptr(m32), int(ld))
        # order with the caller's stream: inputs are ready when the engine's stream runs
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        rc = lib.gsk_engine_submit_ex(self._h, ctypes.byref(r))
        if rc == FULL:
            return False
        _check(rc)
        self._keep[int(tag)] = (A, b, x, val_out, b_out, w_out, m32) + tuple(keep)
        return True

    def submit(self, A, b: torch.Tensor, x: torch.Tensor, tol: float = 1e-8, *, tag: int,
               maxit: Optional[int] = None, breakdown_eps=None,
               stop_weights: Optional[torch.Tensor] = None) -> bool:
        """Admit one (already scaled) system; False if it does not fit now (retry after
        poll())."""
        _vec(b, A.n, "b")
        _vec(x, A.n, "x")
        if stop_weights is not None:
            _vec(stop_weights, A.n, "stop_weights")
        o = _options(maxit, breakdown_eps, stop_weights, None, A.n)
        return self._submit(A, b, x, tol, tag, o, keep=(stop_weights,))

    def submit_gs(self, A, b: torch.Tensor, x: torch.Tensor, p: int = 2, tol: float = 1e-8, *,
                  tag: int, maxit: Optional[int] = None, breakdown_eps=None) -> bool:
        """Admit an unscaled system with a GS(p) stage; the engine scales it in its first chunk
        (outputs allocated here and kept until the system is reported). False if it does not
        fit now."""
        _vec(b, A.n, "b")
        _vec(x, A.n, "x")
        if p < 1:
            raise GskError(ERR_INVALID_ARG, "p must be >= 1")
        src = A.coef if isinstance(A, StencilMatrix) else A.val
        val_out = torch.empty_like(src)
        b_out = torch.empty_like(b)
        w_out = torch.empty_like(b) if p != 2 else None
        o = _options(maxit, breakdown_eps, None, None, A.n)
        return self._submit(A, b, x, tol, tag, o, p, val_out, b_out, w_out)

    def run(self, chunks: int = 1) -> None:
        _check(lib.gsk_engine_run(self._h, int(chunks)))

    def poll(self, wait: bool = True):
        """Results [(tag, Info)] of the systems finished by the last run()."""
        out = (Result * self.max_systems)()
        n = ctypes.c_int32(0)
        _check(lib.gsk_engine_poll(self._h, 1 if wait else 0, out, self.max_systems,
                                   ctypes.byref(n)))
        res = []
        for i in range(n.value):
            tag = int(out[i].tag)
            self._keep.pop(tag, None)
            res.append((tag, _info(out[i].info)))
        if res:
            torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return res

    def usage(self) -> dict:
        u = EngineUsage()
        _check(lib.gsk_engine_get_usage(self._h, ctypes.byref(u)))
        return {"active": u.active, "max_systems": u.max_systems, "max_rows": u.max_rows,
                "free_rows": u.free_rows, "largest_free_rows": u.largest_free_rows}

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib.gsk_engine_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def engine_workspace_bytes(max_rows: int, max_systems: int) -> int:
    return int(lib.gsk_engine_workspace_bytes(int(max_rows), int(max_systems)))


def bicgstab_batch(As, bs, tol: float = 1e-8, *, xs=None, maxit: Optional[int] = None,
                   breakdown_eps=None, check_every: Optional[int] = None):
    """Solve independent systems As[i] x = bs[i] in one batch. Returns (xs, [Info])."""
    count = len(As)
    if count == 0 or len(bs) != count:
        raise ValueError("As and bs must be non-empty and of equal length")
    if xs is None:
        xs = [torch.zeros_like(b) for b in bs]
    for A, b, x in zip(As, bs, xs):
        _vec(b, A.n, "b")
        _vec(x, A.n, "x")
    mats = (Matrix * count)(*[A.c_matrix() for A in As])
    bp = (ctypes.c_void_p * count)(*[b.data_ptr() for b in bs])
    xp = (ctypes.c_void_p * count)(*[x.data_ptr() for x in xs])
    ns = (ctypes.c_int32 * count)(*[A.n for A in As])
    nbytes = int(lib.gsk_bicgstab_batch_workspace_bytes(count, ns))
    ws = _aligned(nbytes, As[0].device)
    o = _options(maxit, breakdown_eps, None, check_every, As[0].n)
    infos = (InfoStruct * count)()
    _check(lib.gsk_bicgstab_batch(count, mats, bp, xp, float(tol), ctypes.byref(o), infos,
                                  *_ws(ws), _stream(As[0].device)))
    return xs, [_info(i) for i in infos]
