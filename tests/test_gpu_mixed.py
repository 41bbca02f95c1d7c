"""Mixed-precision GMRES(m) (FP32 Arnoldi cycles, FP64 restarts) through the C ABI.

Bars: against the oracle's mixed-precision GMRES on the same seeded systems, equal status,
Arnoldi steps within one cycle (m) or 5%, and at tol 1e-10 a solution within 1e-8 of the
oracle's; the FP64 refinement must reach residuals far below float precision; stencil and
CSR operators agree to rounding. At the full 160^3 size the residual of the returned solution
is recomputed independently by the oracle's FP64 product, and GS(p) and the products of the
scaled matrix are compared with the oracle bit for bit on sampled rows.
"""
import numpy as np
import pytest

import oracle
from paper_0812_2769_amd import problems

pytestmark = pytest.mark.gpu


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


def oracle_scaled(P, p=2):
    vo, bo, nrm, w = oracle.gs_scale(P, P.b, p)
    S = P.copy()
    S.val, S.b = vo, bo
    return S, w


def gpu_scaled(G, P, p=2, stencil=True):
    A = G.CsrMatrix.from_problem(P)
    As, bs, _, w = G.gs_scale(A, dev(P.b), p, want_weights=(p != 2))
    M = G.stencil_from_csr(As, *grid_of(P)) if stencil else As
    return M, bs, w


CASES = {
    "slabs_3d_16_gs2": (lambda: problems.slabs_3d(16), 2, 30, 1e-10),
    "slabs_3d_16_gs1": (lambda: problems.slabs_3d(16), 1, 30, 1e-10),
    "checkerboard_3d_32": (lambda: problems.checkerboard_3d(32, blocks_per_axis=4), 2, 30, 1e-8),
    "lap_ragged": (lambda: problems.laplacian((13, 11, 7), conv=(40.0, -25.0, 10.0)), 2, 20,
                   1e-10),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_mixed_matches_oracle(G, case):
    maker, p, m, tol = CASES[case]
    P = maker()
    S, w_o = oracle_scaled(P, p)
    xo, io = oracle.gmres_ir(S, S.b, m=m, tol=tol, weights=None if p == 2 else w_o)
    M, bs, w = gpu_scaled(G, P, p)
    xg, ig = G.gmres_mixed(M, bs, m=m, tol=tol, stop_weights=w)
    assert ig.status == io.status == G.CONVERGED, (ig, io)
    assert abs(ig.iters - io.iters) <= max(m, 0.05 * io.iters), (ig.iters, io.iters)
    assert ig.relres_true < tol
    xg = host(xg)
    cond_bar = 1e-8 if tol <= 1e-10 else 1e-5
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) <= cond_bar


def test_mixed_rounding_sensitive_case_matches_oracle_spread(G):
    """Restarted GMRES on the 2D jump problem is chaotic under rounding: perturbing A at
    float level (relative 2^-23) spreads the oracle's mixed-precision step count over
    478-604 and the GPU's over 401-637, so single runs cannot be compared step for step.
    Both sides solve the same 21 perturbed systems; all must converge and the medians agree
    within 10%. (FP64-ulp perturbations would not do: the FP32 copy of A erases most of them
    on the GPU while the oracle still sees them through its FP64 residual.)"""
    P = problems.square_jump_2d(24)
    S, _ = oracle_scaled(P)
    rng = np.random.default_rng(0)
    it_o, it_g = [], []
    A = G.CsrMatrix.from_problem(P)
    for k in range(21):
        val = S.val if k == 0 else S.val * (1 + 2.0 ** -23 * rng.integers(-2, 3, size=S.val.shape))
        T = S.copy()
        T.val = val
        _, io = oracle.gmres_ir(T, T.b, m=40, tol=1e-8)
        Mg = G.stencil_from_csr(A.with_values(dev(val)), *grid_of(P))
        _, ig = G.gmres_mixed(Mg, dev(T.b), m=40, tol=1e-8)
        assert io.status == ig.status == G.CONVERGED
        it_o.append(io.iters)
        it_g.append(ig.iters)
    assert np.median(it_g) == pytest.approx(np.median(it_o), rel=0.10), (it_g, it_o)


def test_mixed_reaches_fp64_accuracy(G):
    # 1e-13 is far below float precision: only the FP64 residual and update reach it.
    P = problems.laplacian((24, 20, 6), conv=(30.0, 10.0, 5.0))
    M, bs, _ = gpu_scaled(G, P)
    x, info = G.gmres_mixed(M, bs, m=30, tol=1e-13)
    assert info.status == G.CONVERGED and info.relres_true < 1e-13
    S, _ = oracle_scaled(P)
    r = S.b - oracle.spmv(S, host(x))
    assert np.linalg.norm(r) / np.linalg.norm(S.b) < 1e-13


def test_mixed_stencil_and_csr_agree(G):
    # The FP32 copies hold the same values, but the stencil product runs two tiles per
    # workgroup (RPT = 2) and the CSR product one, so the dot products group their partial
    # sums differently: the runs agree to rounding, not bit for bit.
    P = problems.slabs_3d(14)
    Ms, bs, _ = gpu_scaled(G, P, stencil=True)
    Mc, bc, _ = gpu_scaled(G, P, stencil=False)
    xs, i_s = G.gmres_mixed(Ms, bs, m=30, tol=1e-10)
    xc, i_c = G.gmres_mixed(Mc, bc, m=30, tol=1e-10)
    assert i_s.status == i_c.status == G.CONVERGED
    assert abs(i_s.iters - i_c.iters) <= 30
    assert np.linalg.norm(host(xs) - host(xc)) / np.linalg.norm(host(xc)) <= 1e-8


def test_mixed_close_to_fp64_gpu(G):
    P = problems.slabs_3d(20)
    M, bs, _ = gpu_scaled(G, P)
    x64, i64 = G.gmres(M, bs, m=30, tol=1e-10)
    xm, im = G.gmres_mixed(M, bs, m=30, tol=1e-10)
    assert i64.status == im.status == G.CONVERGED
    assert abs(im.iters - i64.iters) <= 30
    assert np.linalg.norm(host(xm) - host(x64)) / np.linalg.norm(host(x64)) <= 1e-8


def test_mixed_workspace_and_errors(G):
    P = problems.slabs_3d(10)
    A = G.CsrMatrix.from_problem(P)
    M = G.stencil_from_csr(A, *grid_of(P))
    n = P.n
    # stencil: equals the generic figure; CSR: holds nnz floats instead of 7 n
    assert G.workspace_bytes_for(M, G.METHOD_GMRES_MIXED, 30) == \
        G.workspace_bytes(G.METHOD_GMRES_MIXED, n, 30)
    assert G.workspace_bytes_for(A, G.METHOD_GMRES_MIXED, 30) > 0
    assert G.workspace_bytes_for(M, G.METHOD_GMRES, 30) == G.workspace_bytes(G.METHOD_GMRES, n, 30)
    full = G.workspace_for(M, G.METHOD_GMRES_MIXED, 30)
    small = full[: full.numel() - 256]
    with pytest.raises(G.GskError) as e:
        G.gmres_mixed(M, dev(P.b), m=30, tol=1e-8, ws=small)
    assert e.value.code == G.ERR_WORKSPACE
    with pytest.raises(G.GskError):
        G.gmres_mixed(M, dev(P.b), m=0, tol=1e-8)


def test_mixed_repeatable(G):
    P = problems.slabs_3d(12)
    M, bs, _ = gpu_scaled(G, P)
    x1, i1 = G.gmres_mixed(M, bs, m=20, tol=1e-10)
    x2, i2 = G.gmres_mixed(M, bs, m=20, tol=1e-10)
    assert (i1.iters, i1.restarts) == (i2.iters, i2.restarts)
    assert np.array_equal(host(x1), host(x2))


@pytest.fixture(scope="module")
def checker160():
    return problems.checkerboard_3d()


def test_checker160_full_size_mixed_vs_fp64(G, checker160):
    """160^3 checkerboard system (n = 4,096,000), GS(2) then GMRES(30), the configuration's
    own workload. Unpreconditioned restarted GMRES(30) needs far more than the paper's
    10,000-step cap to reach 1e-8 here (about 6e-5 after 3,000 steps), so the check runs 20
    cycles: the mixed solver must track FP64 GMRES(30) (true residuals within a factor 2 after
    the same 600 steps), and the residual it reports must equal the FP64 residual of the
    returned solution recomputed independently by the oracle."""
    P = checker160
    M, bs, _ = gpu_scaled(G, P)
    x64, i64 = G.gmres(M, bs, m=30, tol=1e-8, maxit=600)
    xm, im = G.gmres_mixed(M, bs, m=30, tol=1e-8, maxit=600)
    assert i64.status == im.status == G.MAXIT and i64.iters == im.iters == 600
    assert 0.5 < im.relres_true / i64.relres_true < 2.0, (im, i64)
    S, _ = oracle_scaled(P)
    for x, info in ((xm, im), (x64, i64)):
        r = S.b - oracle.spmv(S, host(x))
        rel = np.linalg.norm(r) / np.linalg.norm(S.b)   # x0 = 0
        assert rel == pytest.approx(info.relres_true, rel=1e-6)


def test_checker160_full_size_two_cycles_vs_oracle(G, checker160):
    """160^3 at full size, FP64 GMRES(30) after GS(2), both sides bounded to two cycles (60
    Arnoldi steps): the oracle's orc_gmres on its own scaled system against the HIP solver
    with the stencil operator. Restarted GMRES stagnates here, so, as for the stagnating
    cases of the small parity suite, the first two cycles are compared before rounding has
    been amplified: true residuals to 1e-6 and x to 1e-8 relative."""
    P = checker160
    M, bs, _ = gpu_scaled(G, P)
    x, info = G.gmres(M, bs, m=30, tol=1e-8, maxit=60)
    S, _ = oracle_scaled(P)
    xo, io = oracle.gmres(S, S.b, m=30, tol=1e-8, maxit=60)
    assert info.status == io.status == G.MAXIT and info.iters == io.iters == 60
    assert info.relres_true == pytest.approx(io.relres_true, rel=1e-6)
    np.testing.assert_allclose(host(x), xo, rtol=1e-8, atol=1e-10 * np.abs(xo).max())


def test_checker160_full_size_mixed_two_cycles_vs_oracle(G, checker160):
    """The configuration's own solver at full size: GMRES(30) with FP32 Arnoldi cycles and
    FP64 restarts on the 160^3 system after GS(2), bounded to two cycles (60 Arnoldi steps),
    against the oracle's orc_gmres_ir on its own scaled system. Both store the matrix, the
    basis and w in FP32 and compute in FP64, but the device's sums run in another order, so a
    stored FP32 value can round the other way. Over two cycles that stays near FP32 rounding
    (6e-8; measured 1e-8 on the residual, 7e-8 on x): the bar is 1e-6 relative for both."""
    P = checker160
    M, bs, _ = gpu_scaled(G, P)
    x, info = G.gmres_mixed(M, bs, m=30, tol=1e-8, maxit=60)
    S, _ = oracle_scaled(P)
    xo, io = oracle.gmres_ir(S, S.b, m=30, tol=1e-8, maxit=60)
    rel_res = abs(info.relres_true - io.relres_true) / io.relres_true
    rel_x = np.linalg.norm(host(x) - xo) / np.linalg.norm(xo)
    print(f"mixed 160^3 two cycles: relres {info.relres_true:.6e} vs {io.relres_true:.6e} "
          f"(rel {rel_res:.2e}), x rel {rel_x:.2e}")
    assert info.status == io.status == G.MAXIT and info.iters == io.iters == 60
    assert rel_res < 1e-6
    assert rel_x < 1e-6


def test_checker160_full_size_gs_and_spmv_sampled(G, checker160):
    """The 160^3 system at full size (n = 4,096,000): GS(1) and GS(2) outputs (scaled values,
    right-hand side, row norms, stop weights) and the scaled matrix's product through the CSR
    and the stencil operators, bit for bit equal to the oracle's on 4,000 sampled rows plus
    the first and last. The oracle works on the sampled rows alone."""
    P = checker160
    A = G.CsrMatrix.from_problem(P)
    b = dev(P.b)
    rows = np.sort(np.random.default_rng(11).choice(P.n, size=4000, replace=False))
    rows = np.unique(np.concatenate([rows, [0, P.n - 1]]))
    starts, ends = P.row_ptr[rows], P.row_ptr[rows + 1]
    sel = np.concatenate([np.arange(s, e) for s, e in zip(starts, ends)])
    rp = np.zeros(len(rows) + 1, np.int32)
    rp[1:] = np.cumsum(ends - starts)
    sub = problems.Problem("sub", (len(rows),), rp, P.col_idx[sel].copy(), P.val[sel].copy(),
                           P.b[rows].copy())
    x = np.random.default_rng(12).standard_normal(P.n)
    xd = dev(x)
    for p in (1, 2):
        S, bs, nrm, w = G.gs_scale(A, b, p, want_weights=True)
        vo, bo, n_o, w_o = oracle.gs_scale(sub, sub.b, p)
        np.testing.assert_array_equal(host(S.val)[sel], vo)
        np.testing.assert_array_equal(host(bs)[rows], bo)
        np.testing.assert_array_equal(host(nrm)[rows], n_o)
        np.testing.assert_array_equal(host(w)[rows], w_o)
        Ss = sub.copy()
        Ss.val = vo
        y_o = oracle.spmv(Ss, x)
        np.testing.assert_array_equal(host(G.spmv(S, xd))[rows], y_o)
        St = G.stencil_from_csr(S, *grid_of(P))
        np.testing.assert_array_equal(host(G.spmv(St, xd))[rows], y_o)
        del S, St
