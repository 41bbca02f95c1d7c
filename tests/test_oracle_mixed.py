"""Pins of the oracle's mixed-precision GMRES (iterative refinement with one float-storage
GMRES(m) cycle per correction): the FP64 refinement must deliver FP64 accuracy that float
data alone cannot, the special cases must take the step counts their closed forms give, and
on well-behaved systems the cycle count must stay close to that of FP64 GMRES."""
import numpy as np
import pytest

import oracle
from paper_0812_2769_amd import problems

F32_EPS = 2.0 ** -24


def identity(n, seed):
    rng = np.random.default_rng(seed)
    rp = np.arange(n + 1, dtype=np.int32)
    return problems.Problem("I", (n,), rp, np.arange(n, dtype=np.int32), np.ones(n),
                            rng.standard_normal(n))


def scaled(P, p=2):
    vo, bo, nrm, w = oracle.gs_scale(P, P.b, p)
    S = P.copy()
    S.val, S.b = vo, bo
    return S


def test_identity_takes_two_one_step_cycles():
    # Cycle 1 returns x = beta * fl(b / beta): relative error <= 2^-24 per entry, so the FP64
    # residual is <= 6e-8; cycle 2 repeats the reduction on that residual: <= 4e-15 < 1e-12.
    P = identity(500, 1)
    x, info = oracle.gmres_ir(P, P.b, m=10, tol=1e-12)
    assert info.status == oracle.CONVERGED
    assert info.iters == 2 and info.restarts == 1
    assert np.max(np.abs(x - P.b)) <= 4 * F32_EPS ** 2 * np.max(np.abs(P.b)) * 500


def test_reaches_fp64_accuracy_beyond_float_precision():
    # A relative residual of 1e-13 is far below what float data can represent (6e-8): only
    # the FP64 residual and update can get there. The forward error obeys the usual bound.
    P = scaled(problems.laplacian((12, 10), conv=(40.0, 15.0)))
    x, info = oracle.gmres_ir(P, P.b, m=20, tol=1e-13)
    assert info.status == oracle.CONVERGED and info.relres_true < 1e-13
    A = P.dense()
    xs = np.linalg.solve(A, P.b)
    cond = np.linalg.cond(A)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 10 * cond * 1e-13
    r = P.b - A @ x
    assert np.linalg.norm(r) / np.linalg.norm(P.b) < 1e-13


@pytest.mark.parametrize("maker,m,tol", [
    (lambda: scaled(problems.slabs_3d(12)), 20, 1e-10),
    (lambda: scaled(problems.laplacian((16, 16, 8), conv=(20.0, -10.0, 5.0))), 30, 1e-10),
    (lambda: scaled(problems.square_jump_2d(20)), 40, 1e-8),
])
def test_cycle_count_close_to_fp64(maker, m, tol):
    # Each cycle reduces the residual by a factor far above float precision, so float
    # storage changes the iterates only by rounding: the mixed solve converges in about the
    # same number of Arnoldi steps as FP64 GMRES(m) (one cycle more at most).
    P = maker()
    x64, i64 = oracle.gmres(P, P.b, m=m, tol=tol)
    xir, iir = oracle.gmres_ir(P, P.b, m=m, tol=tol)
    assert i64.status == iir.status == oracle.CONVERGED
    assert abs(iir.iters - i64.iters) <= m, (iir.iters, i64.iters)
    assert iir.relres_true < tol
    # both solutions have relative residual < tol: they differ by at most 2 cond(A) tol
    cond = np.linalg.cond(P.dense())
    assert np.linalg.norm(xir - x64) / np.linalg.norm(x64) <= 2 * cond * tol


def test_first_cycle_matches_float_storage_bound():
    # After one cycle the FP64 residual can fall no further than the float rounding of the
    # data allows: run with a cap of m steps and check that the first cycle's true residual
    # is within a few float ulps' worth of the FP64 cycle's (whichever is larger).
    P = scaled(problems.slabs_3d(10))
    _, i64 = oracle.gmres(P, P.b, m=30, tol=1e-30, maxit=30)
    _, iir = oracle.gmres_ir(P, P.b, m=30, tol=1e-30, maxit=30)
    assert i64.iters == iir.iters == 30
    assert abs(iir.relres_true - i64.relres_true) <= 1e-3 * i64.relres_true + 100 * F32_EPS


def test_edge_cases():
    P = identity(10, 2)
    x, info = oracle.gmres_ir(P, np.zeros(10), m=5, tol=1e-8)
    assert info.status == oracle.CONVERGED and info.iters == 0 and not x.any()
    x, info = oracle.gmres_ir(P, P.b, m=5, tol=1e-8, maxit=0)
    assert info.status == oracle.MAXIT and info.iters == 0
    with pytest.raises(oracle.OracleError):
        oracle.gmres_ir(P, P.b, m=0, tol=1e-8)
