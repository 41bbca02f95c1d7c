"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only, no GPU).

- The oracle (plain C) is built with gcc's sanitizers and runs every routine on small
  convection-diffusion systems (`tests/sanitize/oracle_driver.c`), leak checking on.
- The HIP library is built with the sanitizers on its host code only (each `-fsanitize=` after
  `-Xarch_host`; device code is compiled as usual), and a C driver
  (`tests/sanitize/abi_driver.c`) runs the C ABI's host paths: sizing, configuration checks and
  argument rejection, all of which answer before any device work.

Both builds take about a minute and a half together; they go to a temporary directory.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = os.path.join(HERE, "sanitize")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
CLANG = os.path.join(ROCM, "llvm", "bin", "clang")

pytestmark = pytest.mark.slow


def _run(cmd, env=None, timeout=600):
    p = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    assert p.returncode == 0, (" ".join(cmd), p.stdout[-3000:], p.stderr[-3000:])
    return p.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", exe,
          os.path.join(SAN, "oracle_driver.c"), os.path.join(ROOT, "oracle", "gsk_oracle.c"),
          "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    assert "oracle driver: ok" in _run([exe], env=env)


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)),
                    reason="ROCm compilers not available")
def test_library_host_code_under_asan_ubsan(tmp_path):
    from paper_0812_2769_amd import build
    lib = str(tmp_path / "libgsk_asan.so")
    flags = [f for f in build.HIPCC_FLAGS if f not in ("-O3",)]
    sanitize = []
    for s in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"):
        sanitize += ["-Xarch_host", s]
    _run([HIPCC] + flags + ["-O1", "-g"] + sanitize + ["-o", lib] +
         [os.path.join(build.CSRC, s) for s in build.SOURCES], timeout=900)
    exe = str(tmp_path / "abi_driver")
    _run([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-I", build.INCLUDE, "-o", exe, os.path.join(SAN, "abi_driver.c"),
          "-L", str(tmp_path), "-lgsk_asan", f"-Wl,-rpath,{tmp_path}"])
    # the HIP runtime keeps allocations until exit; leaks are checked on the oracle only
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    assert "abi driver: ok" in _run([exe], env=env)
