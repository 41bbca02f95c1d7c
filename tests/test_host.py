"""Host-side logic that needs no GPU: the workload generators' sizes and recipes, and the
benchmark's argument and traffic-record handling.

The sizes are those of 5/7-point matrices with the Dirichlet neighbours dropped:
nnz = (2d + 1) n - 2 d N^(d-1) for N^d interior nodes.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_0812_2769_amd import problems

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def stencil_nnz(N, d):
    return (2 * d + 1) * N ** d - 2 * d * N ** (d - 1)


def test_benchmark_system_sizes():
    P = problems.square_jump_2d(64)
    assert (P.n, int(P.row_ptr[-1])) == (4096, 20224) == (64 ** 2, stencil_nnz(64, 2))
    P = problems.slabs_3d(80)
    assert (P.n, int(P.row_ptr[-1])) == (512000, 3545600) == (80 ** 3, stencil_nnz(80, 3))
    for N in (12, 17):   # the 160^3 recipe at sizes the CPU suite can afford
        P = problems.checkerboard_3d(N, blocks_per_axis=4)
        assert (P.n, int(P.row_ptr[-1])) == (N ** 3, stencil_nnz(N, 3))


def test_generators_are_seeded():
    a, b = problems.slabs_3d(12, seed=5), problems.slabs_3d(12, seed=5)
    assert np.array_equal(a.val, b.val) and np.array_equal(a.b, b.b)
    c = problems.slabs_3d(12, seed=6)
    assert not np.array_equal(a.val, c.val)


def test_batch_recipe():
    specs = problems.batch_specs(512, seed=1004)
    assert len(specs) == 512
    assert specs == problems.batch_specs(512, seed=1004)
    assert specs != problems.batch_specs(512, seed=1005)
    dims = [s["dims"] for s in specs]
    assert sum(len(d) == 3 for d in dims) == 247
    assert all(len(set(d)) == 1 and 32 <= d[0] <= 96 for d in dims)   # N^d cubes/squares
    assert sum(int(np.prod(d)) for d in dims) == 81830169
    for s in specs[:8]:
        assert 1e2 <= s["jump"] <= 1e6
        assert all(0.0 <= c <= 30.0 for c in s["conv"])
        assert all(0 <= lo <= hi <= 1000 for lo, hi in s["box"])
    P = problems.batch_system(problems.batch_specs(1, seed=3, n_min=10, n_max=10)[0])
    d = len(P.dims)
    assert int(P.row_ptr[-1]) == stencil_nnz(10, d)


def test_bench_runs_on_one_gpu_only():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_record_applies_only_to_its_workload():
    """A counter record applies to its own kernel class, grid and operator only, and only while
    the kernel sources hash to the measured ones (then it scales the algorithmic bytes)."""
    sys.path.insert(0, ROOT)
    import bench
    for rec in bench.TRAFFIC:
        p, g = rec["probe"], rec["grid"]
        bad_grid = 7 if g is None else g + 1
        assert bench.traffic_for(p, bad_grid, "stencil", 1000) is None
        assert bench.traffic_for(p, g, "csr", 1000) is None
        assert bench.traffic_for("gmres_b", g, "stencil", 1000) is None
        assert bench.traffic_for(p, g, "stencil", None) is None
        got = bench.traffic_for(p, g, "stencil", 10 ** 9)
        assert got is None or got == int(rec["ratio"] * 10 ** 9)   # None once sources change
        assert rec["ratio"] is None or 0.9 < rec["ratio"] < 1.2


def test_tuner_rejects_bad_candidates():
    """Candidate shapes are checked before anything runs on the device."""
    from paper_0812_2769_amd import tune
    with pytest.raises(ValueError):
        tune.tune_engine([], shapes=(3,), chunks=(8,))
    with pytest.raises(ValueError):
        tune.tune_engine([], shapes=(1,), chunks=(5,))
    with pytest.raises(ValueError):
        tune.tune_engine([], shapes=(1,), chunks=(0,))
