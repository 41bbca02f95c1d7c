"""Mixed-precision Bi-CGSTAB engines (FP32 storage, FP64 refinement) through the C ABI.

Definition: the oracle's orc_bicgstab_ir. The device sums in a different order and uses fused
multiply-adds, and float-storage Bi-CGSTAB amplifies such differences, so the bars are those
of a rounding-sensitive solver: equal status, the FP64 true residual below tol, iteration
counts within 30% of the oracle's, and x within the conditioning bound. The closed-form case
(A = I: two half steps, one refinement) must match exactly. Within the engine, a system's
result does not depend on what else is in the batch (bit for bit), and repeated runs agree
bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_0812_2769_amd import problems

pytestmark = pytest.mark.gpu
DELTA = 1e-6


@pytest.fixture(scope="module")
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0812_2769_amd import gsk
    return gsk


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def grid_of(P):
    d = list(P.dims) + [1] * (3 - len(P.dims))
    return d[0], d[1], d[2]


def solve(G, items, tol, maxit=10000, rows=None):
    """items: list of (matrix, b, p or 0 for pre-scaled); one engine; returns xs, infos."""
    import torch
    rows = rows or sum((A.n + 511) // 512 * 512 for A, _, _ in items)
    eng = G.Engine(rows, len(items), graph=True, precision="mixed", inner_reduction=DELTA)
    xs = [torch.zeros_like(b) for _, b, _ in items]
    for k, (A, b, p) in enumerate(items):
        ok = (eng.submit_gs(A, b, xs[k], p=p, tol=tol, tag=k, maxit=maxit) if p else
              eng.submit(A, b, xs[k], tol=tol, tag=k, maxit=maxit))
        assert ok
    res = {}
    for _ in range(5000):
        eng.run(1)
        res.update(dict(eng.poll(wait=True)))
        if len(res) == len(items):
            break
    torch.cuda.synchronize()
    eng.close()
    return [host(x) for x in xs], [res[k] for k in range(len(items))]


def oracle_scaled(P, p=2):
    vo, bo, _, w = oracle.gs_scale(P, P.b, p)
    S = P.copy()
    S.val, S.b = vo, bo
    return S, w


def test_identity_two_half_steps(G):
    rng = np.random.default_rng(5)
    n = 700
    rp = np.arange(n + 1, dtype=np.int32)
    P = problems.Problem("I", (n,), rp, np.arange(n, dtype=np.int32), np.ones(n),
                         rng.standard_normal(n))
    A = G.CsrMatrix.from_problem(P)
    xs, infos = solve(G, [(A, dev(P.b), 0)], 1e-12)
    i = infos[0]
    assert i.status == G.CONVERGED and (i.iters, i.restarts, i.half_step) == (2, 1, 1)
    assert np.max(np.abs(xs[0] - P.b)) <= 4 * 2.0 ** -48 * np.max(np.abs(P.b))
    xo, io = oracle.bicgstab_ir(P, P.b, tol=1e-12, delta=DELTA)
    assert (io.iters, io.restarts) == (i.iters, i.restarts)


@pytest.mark.parametrize("seed,p,stencil", [(41, 2, True), (43, 2, False), (47, 1, True)])
def test_mixed_bicgstab_matches_oracle(G, seed, p, stencil):
    P = problems.batch_system(problems.batch_specs(1, seed=seed, n_min=12, n_max=20)[0])
    S, w = oracle_scaled(P, p)
    xo, io = oracle.bicgstab_ir(S, S.b, tol=1e-10, delta=DELTA, weights=None if p == 2 else w)
    A = G.CsrMatrix.from_problem(P)
    M = G.stencil_from_csr(A, *grid_of(P)) if stencil else A
    xs, infos = solve(G, [(M, dev(P.b), p)], 1e-10)
    ig = infos[0]
    assert ig.status == io.status, (ig, io)
    if io.status != G.CONVERGED:
        # float storage diverges on this one (GS(1), 2D jump): both sides end the refinement
        # as stagnated after three steps without progress
        assert io.status == G.STAGNATED and ig.verify_failures == io.verify_failures == 3
        return
    assert ig.relres_true < 1e-10
    assert abs(ig.iters - io.iters) <= 0.3 * io.iters + 5, (ig.iters, io.iters)
    # the scaled system's solution, to the accuracy tol times its condition allows
    x = xs[0]
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 1e-5
    r = S.b - oracle.spmv(S, x)
    rel = np.linalg.norm((w if p != 2 else 1.0) * r) / np.linalg.norm((w if p != 2 else 1.0) * S.b)
    assert rel == pytest.approx(ig.relres_true, rel=1e-6)


def test_mixed_bicgstab_independent_of_batch_and_repeatable(G):
    specs = problems.batch_specs(4, seed=53, n_min=8, n_max=22)
    items = []
    for sp in specs:
        P = problems.batch_system(sp)
        A = G.CsrMatrix.from_problem(P)
        items.append((G.stencil_from_csr(A, *grid_of(P)), dev(P.b), 2))
    xs_all, inf_all = solve(G, items, 1e-9)
    for k in (0, 3):
        xs_one, inf_one = solve(G, [items[k]], 1e-9)
        assert inf_one[0] == inf_all[k]
        assert np.array_equal(xs_one[0], xs_all[k])
    xs_again, inf_again = solve(G, items, 1e-9)
    assert inf_again == inf_all
    assert all(np.array_equal(a, b) for a, b in zip(xs_again, xs_all))


def test_mixed_bicgstab_reaches_fp64_accuracy(G):
    P = problems.laplacian((24, 20, 6), conv=(30.0, 10.0, 5.0))
    A = G.CsrMatrix.from_problem(P)
    M = G.stencil_from_csr(A, *grid_of(P))
    xs, infos = solve(G, [(M, dev(P.b), 2)], 1e-13)
    assert infos[0].status == G.CONVERGED and infos[0].relres_true < 1e-13
    assert infos[0].restarts >= 1
    S, _ = oracle_scaled(P)
    r = S.b - oracle.spmv(S, xs[0])
    assert np.linalg.norm(r) / np.linalg.norm(S.b) < 1e-13
