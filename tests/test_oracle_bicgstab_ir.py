"""Pins of the oracle's mixed-precision Bi-CGSTAB (iterative refinement whose corrections are
Bi-CGSTAB runs with float storage). The closed-form case must take the steps its algebra
gives, the FP64 refinement must reach accuracy that float data cannot, and the measured cost
of float storage on the batch workload's jump problems is recorded (it is why the GPU engine
keeps Bi-CGSTAB in FP64)."""
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
    return S, w


def test_identity_takes_two_half_steps():
    # A = I: p = r~ = fl(b), v = p, alpha = 1, s = r~ - v = 0, so every run ends at its first
    # half step with x += fl(r). Run 1 leaves a residual of at most 2^-24 per entry, run 2
    # squares it: two iterations, one refinement, far below 1e-12.
    P = identity(400, 2)
    x, info = oracle.bicgstab_ir(P, P.b, tol=1e-12)
    assert info.status == oracle.CONVERGED
    assert (info.iters, info.restarts, info.half_step) == (2, 1, 1)
    assert np.max(np.abs(x - P.b)) <= 4 * F32_EPS ** 2 * np.max(np.abs(P.b))


def test_reaches_fp64_accuracy_beyond_float_precision():
    S, _ = scaled(problems.laplacian((12, 10), conv=(40.0, 15.0)))
    x, info = oracle.bicgstab_ir(S, S.b, tol=1e-13, delta=1e-6)
    assert info.status == oracle.CONVERGED and info.relres_true < 1e-13
    assert info.restarts >= 1            # float storage alone cannot get there
    A = S.dense()
    xs = np.linalg.solve(A, S.b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 10 * np.linalg.cond(A) * 1e-13
    assert np.linalg.norm(S.b - A @ x) / np.linalg.norm(S.b) < 1e-13


def test_weights_measure_the_gs2_metric():
    # GS(1) scaling with the weights ||a_i||_1/||a_i||_2 must stop on the same GS(2)-scaled
    # residual as the FP64 solver does: the returned true residual is below tol in that metric.
    P = problems.laplacian((14, 9), conv=(25.0, -10.0))
    S1, w = scaled(P, 1)
    x, info = oracle.bicgstab_ir(S1, S1.b, tol=1e-10, weights=w)
    assert info.status == oracle.CONVERGED
    r = S1.b - S1.dense() @ x
    r0 = np.linalg.norm(w * S1.b)
    assert np.linalg.norm(w * r) / r0 == pytest.approx(info.relres_true, rel=1e-9)
    assert info.relres_true < 1e-10


def test_arguments():
    P = identity(10, 3)
    for d in (0.0, 1.0, -1e-3):
        with pytest.raises(oracle.OracleError):
            oracle.bicgstab_ir(P, P.b, tol=1e-8, delta=d)


def test_float_storage_costs_iterations_on_jump_problems():
    # Measured, not a property of the method: on the batch recipe's jump problems (GS(2),
    # tol 1e-8), float storage with refinement takes clearly more Bi-CGSTAB iterations than
    # FP64 Bi-CGSTAB, more than the 1.9x fewer bytes per iteration could pay for.
    specs = problems.batch_specs(6, seed=1004, n_min=20, n_max=32)
    it64 = itir = 0
    for sp in specs:
        S, _ = scaled(problems.batch_system(sp))
        _, i64 = oracle.bicgstab(S, S.b, tol=1e-8)
        _, iir = oracle.bicgstab_ir(S, S.b, tol=1e-8, delta=1e-6)
        assert i64.status == oracle.CONVERGED
        it64 += i64.iters
        itir += iir.iters
    assert itir > 1.2 * it64, (itir, it64)


def test_divergence_ends_runs_and_stagnates_without_fallback():
    # Float-storage Bi-CGSTAB diverges to overflow on this GS(1)-scaled 2D jump system; the
    # run ends once its estimate exceeds rt / delta, and (with the FP64 continuation switched
    # off) three refinement steps without progress end the solve as stagnated with a finite
    # residual (instead of 10,000 NaN iterations). FP64 Bi-CGSTAB converges on the system.
    P = problems.batch_system(problems.batch_specs(1, seed=47, n_min=12, n_max=20)[0])
    S, w = scaled(P, 1)
    _, i64 = oracle.bicgstab(S, S.b, tol=1e-10, weights=w)
    assert i64.status == oracle.CONVERGED
    _, iir = oracle.bicgstab_ir(S, S.b, tol=1e-10, delta=1e-6, weights=w, fallback=False,
                                run_cap=0)
    assert iir.status == oracle.STAGNATED and iir.verify_failures == 3
    assert np.isfinite(iir.relres_true) and iir.iters < 10000 and iir.fp64_from == 0


@pytest.mark.parametrize("seed,p", [(293, 1), (95, 2), (13, 2)])
def test_fp64_continuation_converges_where_refinement_stops(seed, p):
    # Systems of the batch recipe on which a float-storage run diverges (the true residual is
    # left far above the start, up to overflow; on 95 and 13 refinement alone stagnates): the
    # solve hands over to FP64 Bi-CGSTAB and must end as an FP64 solve does: converged on the
    # GS(2) metric, with the solution dense LU gives (to the condition-number bound) and the
    # reported residual equal to one recomputed here.
    n_min, n_max = 10, 22
    P = problems.batch_system(problems.batch_specs(1, seed=seed, n_min=n_min, n_max=n_max)[0])
    S, w = scaled(P, p)
    W = w if p == 1 else None
    tol = 1e-10 if p == 1 else 1e-8
    if seed != 293:
        _, nofb = oracle.bicgstab_ir(S, S.b, tol=tol, delta=1e-6, weights=W, fallback=False,
                                     run_cap=0)
        assert nofb.status != oracle.CONVERGED
    x, info = oracle.bicgstab_ir(S, S.b, tol=tol, delta=1e-6, weights=W)
    assert info.status == oracle.CONVERGED and info.relres_true < tol
    assert 0 < info.fp64_from < info.iters <= 10000
    A = S.dense()
    xs = np.linalg.solve(A, S.b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 10 * np.linalg.cond(A) * tol
    wt = np.ones(S.n) if W is None else W
    r = wt * (S.b - A @ x)
    assert np.linalg.norm(r) / np.linalg.norm(wt * S.b) == pytest.approx(info.relres_true,
                                                                        rel=1e-6)


def test_undo_restores_the_start_of_a_diverged_run():
    # The continuation starts from the x the refinement last accepted: a run that diverged is
    # undone. On this system the first float run diverges (its estimate rises far above the
    # start before the divergence test ends it), so with maxit at the hand-over point the
    # solve stops with x back at x0 = 0: relative residual exactly 1, not the run's.
    P = problems.batch_system(problems.batch_specs(1, seed=13, n_min=10, n_max=22)[0])
    S, _ = scaled(P)
    _, full = oracle.bicgstab_ir(S, S.b, tol=1e-8, delta=1e-6)
    x, cut = oracle.bicgstab_ir(S, S.b, tol=1e-8, delta=1e-6, maxit=full.fp64_from)
    assert cut.status == oracle.MAXIT and cut.iters == full.fp64_from
    assert cut.relres_true == 1.0 and not x.any()
