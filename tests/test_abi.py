"""The C ABI library loads and exports every symbol include/gsk.h declares; host-side argument
checks reject bad calls before any device work. No GPU needed: nothing here launches a kernel."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsk.h")
LIB = os.path.join(ROOT, "paper_0812_2769_amd", "libgsk.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsk_\w+)\s*\(", text)))


def header_define(name):
    m = re.search(rf"#define\s+{name}\s+\(?(-?\d+)\)?", open(HEADER).read())
    return int(m.group(1))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_0812_2769_amd import build
        build.build()
    from paper_0812_2769_amd import gsk
    return gsk


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert {"gsk_gs_scale", "gsk_gmres", "gsk_bicgstab", "gsk_spmv", "gsk_arnoldi",
            "gsk_workspace_bytes"} <= set(names)
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT\s+(\w+)$", out, flags=re.M))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        getattr(lib.lib, n)


def test_version_and_constants(lib):
    assert lib.lib.gsk_version() == header_define("GSK_VERSION")
    assert lib.MAX_RESTART == header_define("GSK_MAX_RESTART")
    for name, val in (("GSK_ERR_INVALID_ARG", lib.ERR_INVALID_ARG),
                      ("GSK_ERR_ZERO_ROW", lib.ERR_ZERO_ROW),
                      ("GSK_ERR_NONFINITE", lib.ERR_NONFINITE),
                      ("GSK_ERR_WORKSPACE", lib.ERR_WORKSPACE),
                      ("GSK_CONVERGED", lib.CONVERGED), ("GSK_MAXIT", lib.MAXIT),
                      ("GSK_BREAKDOWN", lib.BREAKDOWN), ("GSK_STAGNATED", lib.STAGNATED)):
        assert header_define(name) == val, name


def test_struct_layouts(lib):
    # gsk_csr {int32; int64; 3 pointers}, gsk_options {int32; double; ptr; int32}, gsk_info,
    # gsk_stencil {3 int32; ptr}, gsk_matrix {int32; gsk_csr; gsk_stencil}
    assert ctypes.sizeof(lib.Csr) == 40
    assert ctypes.sizeof(lib.Options) == 32
    assert ctypes.sizeof(lib.InfoStruct) == 48
    assert ctypes.sizeof(lib.Stencil) == 24
    assert ctypes.sizeof(lib.Matrix) == 72
    assert lib.Matrix.csr.offset == 8 and lib.Matrix.stencil.offset == 48


def test_defaults(lib):
    o = lib.default_options()
    assert o.maxit == 10000
    assert o.breakdown_eps == pytest.approx(1e-16 * 2.220446049250313e-16, rel=1e-15)
    assert o.check_every == 8 and not o.stop_weights


def test_workspace_bytes(lib):
    n = 512000
    g30 = lib.workspace_bytes(lib.METHOD_GMRES, n, 30)
    g20 = lib.workspace_bytes(lib.METHOD_GMRES, n, 20)
    assert g30 - g20 == 10 * 8 * ((n + 63) // 64 * 64)
    assert lib.workspace_bytes(lib.METHOD_BICGSTAB, n) > 7 * 8 * n
    assert lib.workspace_bytes(lib.METHOD_GS, n) > 0
    assert lib.workspace_bytes(lib.METHOD_GMRES, n, 0) == 0
    assert lib.workspace_bytes(lib.METHOD_GMRES, n, 65) == 0
    assert lib.workspace_bytes(lib.METHOD_GMRES, 0, 10) == 0
    assert lib.workspace_bytes(99, n, 10) == 0


def _fake_csr(lib, n=10, nnz=30):
    # non-NULL placeholders: every call below is rejected before any device access
    return lib.Csr(n, nnz, 0x1000, 0x2000, 0x3000)


def _fake_matrix(lib, n=10, nnz=30):
    return lib.Matrix(lib.MATRIX_CSR, _fake_csr(lib, n, nnz), lib.Stencil(0, 0, 0, None))


def test_host_side_rejections(lib):
    L = lib.lib
    c = _fake_csr(lib)
    mtx = _fake_matrix(lib)
    info = lib.InfoStruct()
    o = lib.default_options()
    ws_ok = 0x100000  # 256-aligned placeholder, paired with too small a size below
    # NULL matrix
    assert L.gsk_gs_scale(None, 0x10, 2, 0x20, 0x30, None, None, ws_ok, 1 << 30, None) == -1
    assert b"NULL" in L.gsk_last_error()
    # p < 1
    assert L.gsk_gs_scale(ctypes.byref(c), 0x10, 0, 0x20, 0x30, None, None, ws_ok, 1 << 30, None) == -1
    # bad n / nnz
    bad = lib.Matrix(lib.MATRIX_CSR, lib.Csr(0, 0, 0x1000, 0, 0), lib.Stencil(0, 0, 0, None))
    assert L.gsk_spmv(ctypes.byref(bad), 0x10, 0x20, None) == -1
    bad = lib.Matrix(lib.MATRIX_CSR, lib.Csr(5, -1, 0x1000, 0x2000, 0x3000),
                     lib.Stencil(0, 0, 0, None))
    assert L.gsk_spmv(ctypes.byref(bad), 0x10, 0x20, None) == -1
    # stencil matrices: grid too small, NULL planes, unknown kind
    bad = lib.Matrix(lib.MATRIX_STENCIL, lib.Csr(0, 0, None, None, None), lib.Stencil(1, 4, 4, 0x10))
    assert L.gsk_spmv(ctypes.byref(bad), 0x10, 0x20, None) == -1
    bad = lib.Matrix(lib.MATRIX_STENCIL, lib.Csr(0, 0, None, None, None), lib.Stencil(4, 4, 4, None))
    assert L.gsk_spmv(ctypes.byref(bad), 0x10, 0x20, None) == -1
    bad = lib.Matrix(7, lib.Csr(0, 0, None, None, None), lib.Stencil(4, 4, 4, 0x10))
    assert L.gsk_spmv(ctypes.byref(bad), 0x10, 0x20, None) == -1
    # stencil packing: grid does not match n
    assert L.gsk_stencil_from_csr(ctypes.byref(c), 3, 3, 1, 0x40, ws_ok, 1 << 30, None) == -1
    # restart length out of range
    assert L.gsk_gmres(ctypes.byref(mtx), 0x10, 0x20, 0, 1e-8, None, ctypes.byref(info), ws_ok,
                       1 << 30, None) == -1
    assert L.gsk_gmres(ctypes.byref(mtx), 0x10, 0x20, 65, 1e-8, None, ctypes.byref(info), ws_ok,
                       1 << 30, None) == -1
    # tol <= 0, maxit < 0, check_every out of range
    assert L.gsk_bicgstab(ctypes.byref(mtx), 0x10, 0x20, 0.0, None, ctypes.byref(info), ws_ok,
                          1 << 30, None) == -1
    o.maxit = -1
    assert L.gsk_bicgstab(ctypes.byref(mtx), 0x10, 0x20, 1e-8, ctypes.byref(o), ctypes.byref(info),
                          ws_ok, 1 << 30, None) == -1
    o = lib.default_options()
    o.check_every = 0
    assert L.gsk_bicgstab(ctypes.byref(mtx), 0x10, 0x20, 1e-8, ctypes.byref(o), ctypes.byref(info),
                          ws_ok, 1 << 30, None) == -1
    # workspace: NULL, misaligned, too small
    assert L.gsk_bicgstab(ctypes.byref(mtx), 0x10, 0x20, 1e-8, None, ctypes.byref(info), None,
                          1 << 30, None) == -4
    assert L.gsk_bicgstab(ctypes.byref(mtx), 0x10, 0x20, 1e-8, None, ctypes.byref(info), ws_ok + 8,
                          1 << 30, None) == -4
    assert L.gsk_gmres(ctypes.byref(mtx), 0x10, 0x20, 10, 1e-8, None, ctypes.byref(info), ws_ok, 16,
                       None) == -4
    assert b"needed" in L.gsk_last_error()
    # arnoldi: ldv < n
    steps = ctypes.c_int32(0)
    assert L.gsk_arnoldi(ctypes.byref(mtx), 0x10, 4, 0x20, 5, 0x30, ctypes.byref(steps), ws_ok,
                         1 << 30, None) == -1


def test_binding_refuses_cpu_tensors(lib):
    import torch
    with pytest.raises(ValueError):
        lib.CsrMatrix(torch.zeros(3, dtype=torch.int32), torch.zeros(2, dtype=torch.int32),
                      torch.zeros(2, dtype=torch.float64))
    # workspaces and optional outputs must be device memory too (a host pointer handed to a
    # kernel would fault the GPU)
    with pytest.raises(ValueError):
        lib._ws(torch.zeros(1024, dtype=torch.uint8))
    with pytest.raises(ValueError):
        lib._opt_vec(torch.zeros(3, dtype=torch.float64), 3, "weights")
    assert lib._opt_vec(None, 3, "weights") is None


def test_engine_struct_layouts_and_rejections(lib):
    # gsk_result {int64; gsk_info}, gsk_engine_usage {2 int32; 3 int64}
    assert ctypes.sizeof(lib.Result) == 56
    assert ctypes.sizeof(lib.EngineUsage) == 32
    L = lib.lib
    assert lib.engine_workspace_bytes(0, 4) == 0
    assert lib.engine_workspace_bytes(1000, 0) == 0
    assert lib.engine_workspace_bytes(1 << 20, 64) > 7 * 8 * (1 << 20)
    h = ctypes.c_void_p()
    # graph mode needs a non-default stream and an even check_every; sizes must be positive
    assert L.gsk_engine_create(0x100000, 1 << 30, 1000, 4, 8, lib.ENGINE_GRAPH, None,
                               ctypes.byref(h)) == -1
    assert L.gsk_engine_create(0x100000, 1 << 30, 0, 4, 8, 0, None, ctypes.byref(h)) == -1
    assert L.gsk_engine_create(0x100000, 1 << 30, 1000, 4, 0, 0, None, ctypes.byref(h)) == -1
    assert L.gsk_engine_create(0x100000, 16, 1000, 4, 8, 0, None, ctypes.byref(h)) == -4
    assert L.gsk_engine_create(None, 1 << 30, 1000, 4, 8, 0, None, ctypes.byref(h)) == -4
    n = ctypes.c_int32(0)
    assert L.gsk_engine_poll(None, 1, None, 0, ctypes.byref(n)) == -1
    assert L.gsk_engine_run(None, 1) == -1
    assert L.gsk_engine_destroy(None) == 0
    ns = (ctypes.c_int32 * 2)(300, 0)
    assert L.gsk_bicgstab_batch_workspace_bytes(2, ns) == 0
    ns = (ctypes.c_int32 * 2)(300, 100)
    assert L.gsk_bicgstab_batch_workspace_bytes(2, ns) == lib.engine_workspace_bytes(768, 2)


def test_struct_layouts_match_the_header(lib, tmp_path):
    """sizeof and field offsets of every ABI struct, from a C program compiled against
    include/gsk.h, equal those of the ctypes binding."""
    checks = {
        "gsk_csr": (lib.Csr, ["n", "nnz", "row_ptr", "col_idx", "val"]),
        "gsk_options": (lib.Options, None),
        "gsk_info": (lib.InfoStruct, None),
        "gsk_matrix": (lib.Matrix, None),
        "gsk_result": (lib.Result, ["tag", "info"]),
        "gsk_engine_usage": (lib.EngineUsage, ["active", "max_systems", "max_rows",
                                               "free_rows", "largest_free_rows"]),
        "gsk_engine_config": (lib.EngineConfig, ["max_rows", "max_systems", "method", "m",
                                                 "precision", "check_every", "flags",
                                                 "tile_units", "inner_reduction", "run_cap",
                                                 "class_shapes"]),
        "gsk_engine_request": (lib.EngineRequest, ["A", "b", "x", "tol", "opt", "tag", "gs_p",
                                                   "val_out", "b_out", "stop_weight_out",
                                                   "mat32", "mat32_ld"]),
    }
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "gsk.h"', "int main(void) {"]
    for cname, (_, fields) in checks.items():
        src.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for f in fields or []:
            src.append(f'  printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    src += ["  return 0;", "}"]
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(c), "-o", str(exe)],
                   check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True,
                                                       text=True, check=True).stdout.split("\n")
               if line)
    for cname, (ct, fields) in checks.items():
        assert int(got[cname]) == ctypes.sizeof(ct), cname
        for f in fields or []:
            assert int(got[f"{cname}.{f}"]) == getattr(ct, f).offset, (cname, f)


def test_engine_config_rejections(lib):
    L = lib.lib
    good = lib.EngineConfig(4096, 4, lib.METHOD_GMRES, 20, lib.PRECISION_MIXED, 8, 0, 0, 0.0)
    assert L.gsk_engine_workspace_bytes_ex(ctypes.byref(good)) > 0
    bad = [
        lib.EngineConfig(4096, 4, lib.METHOD_GMRES, 0, 0, 8, 0, 0, 0.0),      # m = 0
        lib.EngineConfig(4096, 4, lib.METHOD_GMRES, 65, 0, 8, 0, 0, 0.0),     # m > 64
        lib.EngineConfig(4096, 4, lib.METHOD_ARNOLDI, 20, 0, 8, 0, 0, 0.0),   # method
        lib.EngineConfig(4096, 4, lib.METHOD_BICGSTAB, 0, 0, 0, 0, 0, 0.0),   # check_every
        lib.EngineConfig(4096, 4, lib.METHOD_BICGSTAB, 0, 1, 8, 0, 0, 1.5),   # reduction
        lib.EngineConfig(4096, 4, lib.METHOD_GMRES, 20, 0, 8, 0, 2, 0.0),     # 2 tiles, GMRES
        lib.EngineConfig(4096, 4, lib.METHOD_BICGSTAB, 0, 1, 8, 0, 2, 0.0),   # 2 tiles, mixed
        lib.EngineConfig(0, 4, lib.METHOD_BICGSTAB, 0, 0, 8, 0, 0, 0.0),      # no rows
        lib.EngineConfig(4096, 4, lib.METHOD_BICGSTAB, 0, 7, 8, 0, 0, 0.0),   # precision
        # per-class shapes: FP64 Bi-CGSTAB only, codes 0..3, three classes
        lib.EngineConfig(4096, 4, lib.METHOD_GMRES, 20, 0, 8, 0, 0, 0.0, 0, 0x3),
        lib.EngineConfig(4096, 4, lib.METHOD_BICGSTAB, 0, 1, 8, 0, 0, 0.0, 0, 0x3),
        lib.EngineConfig(4096, 4, lib.METHOD_BICGSTAB, 0, 0, 8, 0, 0, 0.0, 0, 0x4),
        lib.EngineConfig(4096, 4, lib.METHOD_BICGSTAB, 0, 0, 8, 0, 0, 0.0, 0, 0x1000),
    ]
    h = ctypes.c_void_p()
    for cfg in bad:
        assert L.gsk_engine_workspace_bytes_ex(ctypes.byref(cfg)) == 0
        assert L.gsk_engine_create_ex(ctypes.byref(cfg), 0x100000, 1 << 30, None,
                                      ctypes.byref(h)) == lib.ERR_INVALID_ARG
    assert L.gsk_engine_create_ex(None, 0x100000, 1 << 30, None, ctypes.byref(h)) == \
        lib.ERR_INVALID_ARG
    # per-class shapes hand out rows in pairs of tiles and keep one unit list per class
    one = lib.EngineConfig(4096, 4, lib.METHOD_BICGSTAB, 0, 0, 8, 0, 0, 0.0, 0, 0)
    three = lib.EngineConfig(4096, 4, lib.METHOD_BICGSTAB, 0, 0, 8, 0, 0, 0.0, 0, 0x321)
    assert L.gsk_engine_workspace_bytes_ex(ctypes.byref(three)) >= \
        L.gsk_engine_workspace_bytes_ex(ctypes.byref(one)) > 0
    # a valid configuration with too small a workspace fails before any device work
    assert L.gsk_engine_create_ex(ctypes.byref(good), 0x100000, 256, None,
                                  ctypes.byref(h)) == lib.ERR_WORKSPACE


def test_stream_mix_sizes_and_rejections(lib):
    """The measurement hook sizes its buffer and rejects bad arguments before any device work."""
    L = lib.lib
    n = 1000
    tiles = (n + 255) // 256
    assert L.gsk_stream_mix_bytes(11, 2, n) == 8 * (13 * n + (tiles + 7) // 8 * 8)
    assert L.gsk_stream_mix_bytes(1, 0, n) == 8 * (n + 8)
    assert L.gsk_stream_mix_bytes(2, 2, n) == 0
    assert L.gsk_stream_mix_bytes(11, 2, 0) == 0
    ms = ctypes.c_float(0.0)
    assert L.gsk_stream_mix_ms(2, 2, n, 0x100000, 1 << 20, 1, ctypes.byref(ms), None) == \
        lib.ERR_INVALID_ARG
    assert L.gsk_stream_mix_ms(11, 2, n, 0x100000, 64, 1, ctypes.byref(ms), None) == \
        lib.ERR_WORKSPACE
    assert L.gsk_stream_mix_ms(11, 2, n, 0x100000, 1 << 20, 0, ctypes.byref(ms), None) == \
        lib.ERR_INVALID_ARG
    assert L.gsk_stream_mix_ms(11, 2, n, 0x100000, 1 << 20, 1001, ctypes.byref(ms), None) == \
        lib.ERR_INVALID_ARG
