"""Build the HIP library libgsk.so (gfx950) in-tree with hipcc.

Run `python -m paper_0812_2769_amd.build` (or call build()) after changing any source under
csrc/. Nothing here runs on the GPU.
"""
import concurrent.futures
import os
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libgsk.so")
SOURCES = ["api.hip", "gs_spmv.hip", "gmres.hip", "bicgstab.hip", "batch.hip", "batch_gmres.hip",
           "batch_mixed.hip", "measure.hip"]
ARCH = "gfx950"

COMPILE_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE,
    "-I", CSRC,
]
LINK_FLAGS = [
    f"--offload-arch={ARCH}",
    "-shared",
    # roctx ranges for rocprofv3's marker trace
    "-L", os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib"),
    "-lrocprofiler-sdk-roctx",
]
# Flags of a one-command build (every source compiled and linked by one hipcc call).
HIPCC_FLAGS = COMPILE_FLAGS + LINK_FLAGS[1:]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose: bool = False, extra=None) -> str:
    """Compiles every source to an object in parallel (the translation units share no device
    code), then links libgsk.so; the library is replaced only when every step succeeded."""
    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with tempfile.TemporaryDirectory(prefix="gsk_build_") as tmpdir:
        cmds = []
        for s in SOURCES:
            obj = os.path.join(tmpdir, os.path.splitext(s)[0] + ".o")
            cmds.append((obj, [hipcc()] + COMPILE_FLAGS + list(extra or []) +
                         ["-c", "-o", obj, os.path.join(CSRC, s)]))
        if verbose:
            for _, c in cmds:
                print(" ".join(c), flush=True)
        with concurrent.futures.ThreadPoolExecutor(jobs) as pool:
            done = list(pool.map(lambda c: subprocess.run(c[1]).returncode, cmds))
        failed = [s for s, rc in zip(SOURCES, done) if rc != 0]
        if failed:
            raise RuntimeError(f"hipcc failed on {', '.join(failed)}")
        tmp = LIB + ".tmp"
        link = [hipcc()] + LINK_FLAGS + list(extra or []) + ["-o", tmp] + [o for o, _ in cmds]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.run(link, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
