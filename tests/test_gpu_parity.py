"""HIP path (through the C ABI) against the FP64 oracle, element by element.

Bars: integer-valued SpMV and every SpMV/GS(p<=2) result bit-exact (both sum each row in
storage order with rounded products and divide/sqrt correctly rounded); GS(p>2) within 1e-13
(pow may differ by an ulp); Arnoldi basis and Hessenberg entries within 1e-11 relative (only
the summation order of the dot products differs); solver iteration counts within 5% (or 1),
equal status, and at a 1e-10 residual tolerance a solution within 1e-8 of the oracle's.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_0812_2769_amd import problems

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0812_2769_amd import gsk
    return gsk


def up(G, P):
    import torch
    return G.CsrMatrix.from_problem(P), torch.from_numpy(np.ascontiguousarray(P.b)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def oracle_scaled(P, p):
    vo, bo, nrm, w = oracle.gs_scale(P, P.b, p)
    S = P.copy()
    S.val, S.b = vo, bo
    return S, nrm, w


def with_empty_rows(n, seed):
    P = problems.random_sparse(n, 4, seed)
    rng = np.random.default_rng(seed)
    keep_rows = rng.random(n) > 0.2
    rows = np.repeat(np.arange(n), np.diff(P.row_ptr))
    keep = keep_rows[rows]
    counts = np.bincount(rows[keep], minlength=n)
    rp = np.zeros(n + 1, np.int32)
    rp[1:] = np.cumsum(counts)
    return problems.Problem("empty_rows", (n,), rp, P.col_idx[keep].copy(), P.val[keep].copy(),
                            P.b.copy())


SPMV_CASES = {
    "random_real": lambda: problems.random_sparse(3000, 5, 1),
    "random_int": lambda: problems.random_sparse(2000, 6, 2, integer=True),
    "long_rows": lambda: problems.random_sparse(700, 40, 3, max_row=600),
    "n1": lambda: problems.random_sparse(1, 1, 4),
    "ragged257": lambda: problems.random_sparse(257, 7, 5),
    "empty_rows": lambda: with_empty_rows(1500, 6),
    "stencil3d": lambda: problems.slabs_3d(14),
    "stencil2d": lambda: problems.square_jump_2d(33),
}


@pytest.mark.parametrize("case", sorted(SPMV_CASES))
def test_spmv_bitwise(G, case):
    import torch
    P = SPMV_CASES[case]()
    A, _ = up(G, P)
    rng = np.random.default_rng(99)
    x = rng.standard_normal(P.n)
    if case == "random_int":
        x = rng.integers(-9, 10, size=P.n).astype(float)
    y = G.spmv(A, torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(y), oracle.spmv(P, x))


GS_CASES = {
    "random": lambda: problems.random_sparse(2500, 5, 11),
    "long_rows": lambda: problems.random_sparse(600, 30, 12, max_row=500),
    "square_jump_2d_40": lambda: problems.square_jump_2d(40),
    "slabs_3d_20": lambda: problems.slabs_3d(20),
    "problem4": lambda: problems.problem4(12, 1e6),
    "ragged": lambda: problems.random_sparse(1031, 3, 13),
}


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("case", sorted(GS_CASES))
def test_gs_scale_parity(G, case, p):
    P = GS_CASES[case]()
    A, b = up(G, P)
    S, bs, nrm, w = G.gs_scale(A, b, p, want_weights=True)
    vo, bo, n_o, w_o = oracle.gs_scale(P, P.b, p)
    got = [host(S.val), host(bs), host(nrm), host(w)]
    want = [vo, bo, n_o, w_o]
    for g, o in zip(got, want):
        if p <= 2:
            np.testing.assert_array_equal(g, o)
        else:
            np.testing.assert_allclose(g, o, rtol=1e-13, atol=0)


def test_gs_scale_in_place(G):
    P = problems.square_jump_2d(20)
    A, b = up(G, P)
    S, bs, _, _ = G.gs_scale(A, b, 2, inplace=True)
    assert S.val.data_ptr() == A.val.data_ptr() and bs.data_ptr() == b.data_ptr()
    vo, bo, _, _ = oracle.gs_scale(P, P.b, 2)
    np.testing.assert_array_equal(host(A.val), vo)
    np.testing.assert_array_equal(host(b), bo)


def test_gs_scale_errors(G):
    import torch
    P = problems.random_sparse(600, 4, 21)
    Z = P.copy()
    Z.val[Z.row_ptr[300]:Z.row_ptr[301]] = 0.0
    A, b = up(G, Z)
    with pytest.raises(G.GskError) as e:
        G.gs_scale(A, b, 2)
    assert e.value.code == G.ERR_ZERO_ROW
    N = P.copy()
    N.val[17] = np.nan
    A, b = up(G, N)
    with pytest.raises(G.GskError) as e:
        G.gs_scale(A, b, 1)
    assert e.value.code == G.ERR_NONFINITE
    # a column index out of range is caught by the device-side structure check, before any
    # indexed access
    Bad = P.copy()
    Bad.col_idx = Bad.col_idx.copy()
    Bad.col_idx[5] = P.n + 3
    A, b = up(G, Bad)
    with pytest.raises(G.GskError) as e:
        G.gs_scale(A, b, 2)
    assert e.value.code == G.ERR_INVALID_ARG
    # row_ptr[n] != nnz
    A, b = up(G, P)
    A2 = G.CsrMatrix(A.row_ptr.clone(), A.col_idx, A.val)
    A2.row_ptr[-1] = P.nnz - 1
    torch.cuda.synchronize()
    with pytest.raises(G.GskError) as e:
        G.gs_scale(A2, b, 2)
    assert e.value.code == G.ERR_INVALID_ARG


@pytest.mark.parametrize("m", [1, 7, 20, 33])
def test_arnoldi_parity(G, m):
    import torch
    S, _, _ = oracle_scaled(problems.square_jump_2d(24), 2)
    A, b = up(G, S)
    V, H, k = G.arnoldi(A, b, m)
    torch.cuda.synchronize()
    Vo, Ho, ko = oracle.arnoldi(S, S.b, m)
    assert k == ko == m
    V, H = host(V), host(H)
    assert np.abs(H - Ho).max() <= 1e-11 * np.abs(Ho).max()
    assert np.abs(V[:, :k + 1] - Vo[:, :k + 1]).max() <= 1e-11
    VtV = V[:, :k + 1].T @ V[:, :k + 1]
    assert np.abs(VtV - np.eye(k + 1)).max() < 1e-13


def _check_solver(info, o_info, x, x_o, tol, sol_rtol):
    assert info.status == o_info.status, (info, o_info)
    assert abs(info.iters - o_info.iters) <= max(1, 0.05 * o_info.iters), (info, o_info)
    if o_info.status == oracle.CONVERGED:
        assert info.relres_true < tol
        err = np.linalg.norm(x - x_o) / np.linalg.norm(x_o)
        assert err <= sol_rtol, err
    else:
        assert info.relres_true == pytest.approx(o_info.relres_true, rel=0.05)


SOLVE_CASES = {
    # name: (problem maker, p, m, tol, bicgstab_sensitive)
    "slabs_3d_16_gs2": (lambda: problems.slabs_3d(16), 2, 30, 1e-10, False),
    "slabs_3d_16_gs1": (lambda: problems.slabs_3d(16, seed=5), 1, 30, 1e-10, False),
    "c1_24_gs2": (lambda: problems.square_jump_2d(24), 2, 20, 1e-10, False),
    "p4_10": (lambda: problems.problem4(10, 1e4), 2, 10, 1e-4, True),
    "lap_conv_ragged": (lambda: problems.laplacian((37, 29), conv=(15.0, -7.0)), 2, 15, 1e-10,
                        True),
    "p1_32": (lambda: problems.problem1(32), 2, 10, 1e-7, False),
}


def _perturbed_medians(G, S, p, tol, weights_np, weights_dev, count=31):
    """Bi-CGSTAB's iteration count on some problems moves by several percent under 1-ulp
    changes of the data (its residual is irregular and rounding is amplified; the oracle
    alone spans 73-80 iterations on lap_conv_ragged over 200 such perturbations, and on the
    indefinite Problem 4 system it breaks down in 2 of 300). There the parity bar applies to
    the same `count` perturbed systems on both sides: at least 80% converge on each side and
    the medians of the converged runs' iteration counts agree within 5%."""
    import torch
    g_it, o_it = [], []
    A = G.CsrMatrix.from_problem(S)
    for k in range(count):
        rng = np.random.default_rng(1000 + k)
        T = S.copy()
        T.val = S.val * (1 + 2.2e-16 * rng.choice([-1, 0, 1], size=S.nnz))
        T.b = S.b * (1 + 2.2e-16 * rng.choice([-1, 0, 1], size=S.n))
        Ad = A.with_values(torch.from_numpy(T.val).cuda())
        x, gi = G.bicgstab(Ad, torch.from_numpy(T.b).cuda(), tol=tol, stop_weights=weights_dev)
        xo, oi = oracle.bicgstab(T, T.b, tol=tol, weights=weights_np)
        if gi.status == oracle.CONVERGED:
            assert gi.relres_true < tol
            g_it.append(gi.iters)
        if oi.status == oracle.CONVERGED:
            o_it.append(oi.iters)
    assert len(g_it) >= 0.8 * count and len(o_it) >= 0.8 * count, (len(g_it), len(o_it))
    return float(np.median(g_it)), float(np.median(o_it))


@pytest.mark.parametrize("case", sorted(SOLVE_CASES))
def test_bicgstab_parity(G, case):
    import torch
    maker, p, m, tol, sensitive = SOLVE_CASES[case]
    P = maker()
    S, nrm, w = oracle_scaled(P, p)
    A, b = up(G, P)
    As, bs, _, wd = G.gs_scale(A, b, p, want_weights=True)
    weights = wd if p != 2 else None
    x, info = G.bicgstab(As, bs, tol=tol, stop_weights=weights)
    torch.cuda.synchronize()
    x_o, o_info = oracle.bicgstab(S, S.b, tol=tol, weights=None if p == 2 else w)
    if not sensitive:
        _check_solver(info, o_info, host(x), x_o, tol, 1e-8 if tol <= 1e-10 else 1e-4)
        return
    assert info.status == o_info.status == oracle.CONVERGED and info.relres_true < tol
    g_med, o_med = _perturbed_medians(G, S, p, tol, None if p == 2 else w, weights)
    assert abs(g_med - o_med) <= max(1, 0.05 * o_med), (g_med, o_med)


@pytest.mark.parametrize("case", sorted(SOLVE_CASES))
def test_gmres_parity(G, case):
    import torch
    maker, p, m, tol, _ = SOLVE_CASES[case]
    P = maker()
    S, nrm, w = oracle_scaled(P, p)
    A, b = up(G, P)
    As, bs, _, wd = G.gs_scale(A, b, p, want_weights=True)
    weights = wd if p != 2 else None
    x, info = G.gmres(As, bs, m=m, tol=tol, stop_weights=weights, maxit=3000)
    torch.cuda.synchronize()
    x_o, o_info = oracle.gmres(S, S.b, m=m, tol=tol, weights=None if p == 2 else w, maxit=3000)
    if o_info.status == oracle.CONVERGED:
        _check_solver(info, o_info, host(x), x_o, tol, 1e-8 if tol <= 1e-10 else 1e-4)
        return
    # Restarted GMRES that stagnates (Table 1's observation): the level it wanders at after
    # thousands of steps is not reproducible under rounding (the oracle alone spans 3e-7 to
    # 7e-5 on c1_24_gs2 under 1-ulp perturbations of the data). Both sides must stagnate, and
    # the first two cycles -- before rounding has been amplified -- must agree closely.
    assert info.status == o_info.status, (info, o_info)
    assert info.iters == o_info.iters
    x2, i2 = G.gmres(As, bs, m=m, tol=tol, stop_weights=weights, maxit=2 * m)
    torch.cuda.synchronize()
    x2o, i2o = oracle.gmres(S, S.b, m=m, tol=tol, weights=None if p == 2 else w, maxit=2 * m)
    assert i2.iters == i2o.iters == 2 * m
    assert i2.relres_true == pytest.approx(i2o.relres_true, rel=1e-6)
    np.testing.assert_allclose(host(x2), x2o, rtol=1e-8, atol=1e-10 * np.abs(x2o).max())


def test_gmres_stagnation_matches(G):
    # GMRES(20) stagnates on the 2D jump problem (the paper's observation for restarted
    # GMRES, Table 1); both sides end at the cap with the same residual level.
    import torch
    P = problems.square_jump_2d(32)
    S, _, _ = oracle_scaled(P, 2)
    A, b = up(G, S)
    x, info = G.gmres(A, b, m=20, tol=1e-8, maxit=600)
    torch.cuda.synchronize()
    x_o, o_info = oracle.gmres(S, S.b, m=20, tol=1e-8, maxit=600)
    assert info.status == o_info.status == oracle.MAXIT
    assert info.iters == o_info.iters == 600
    assert info.relres_true == pytest.approx(o_info.relres_true, rel=1e-3)


def _dense(A, b):
    n = A.shape[0]
    rp, ci, v = [0], [], []
    for i in range(n):
        nz = np.nonzero(A[i])[0]
        ci += list(nz)
        v += list(A[i, nz])
        rp.append(len(ci))
    return problems.Problem("d", (n,), np.array(rp, np.int32), np.array(ci, np.int32),
                            np.array(v, float), np.asarray(b, float))


def test_edge_cases(G):
    import torch
    # identity: GMRES one step, Bi-CGSTAB a half step
    P = _dense(np.eye(300), np.arange(1.0, 301.0))
    A, b = up(G, P)
    x, info = G.gmres(A, b, m=5, tol=1e-12)
    assert info.status == G.CONVERGED and info.iters == 1
    np.testing.assert_allclose(host(x), P.b, rtol=1e-15)
    x, info = G.bicgstab(A, b, tol=1e-12)
    assert info.status == G.CONVERGED and info.iters == 1 and info.half_step == 1
    # rotation: GMRES exact in 2 steps, Bi-CGSTAB breaks down at once
    R = _dense(np.array([[0.0, 1.0], [-1.0, 0.0]]), [1.0, 0.0])
    A, b = up(G, R)
    x, info = G.gmres(A, b, m=5, tol=1e-12)
    assert info.status == G.CONVERGED and info.iters == 2
    np.testing.assert_allclose(host(x), [0.0, 1.0], atol=1e-15)
    x, info = G.bicgstab(A, b, tol=1e-12)
    assert info.status == G.BREAKDOWN and info.iters == 0
    assert info.breakdown_test == G.BRK_SIGMA
    _, o_info = oracle.bicgstab(R, R.b, tol=1e-12)
    assert o_info.breakdown_test == info.breakdown_test
    # zero right-hand side: x0 = 0 is exact
    S, _, _ = oracle_scaled(problems.square_jump_2d(12), 2)
    A, b = up(G, S)
    z = torch.zeros_like(b)
    for solve in (lambda **k: G.gmres(A, z, m=10, **k), lambda **k: G.bicgstab(A, z, **k)):
        x, info = solve()
        assert info.status == G.CONVERGED and info.iters == 0
        assert torch.count_nonzero(x).item() == 0
    # maxit = 0 and maxit = 1
    for solve, osolve in ((lambda **k: G.gmres(A, b, m=10, **k),
                           lambda **k: oracle.gmres(S, S.b, m=10, **k)),
                          (lambda **k: G.bicgstab(A, b, **k),
                           lambda **k: oracle.bicgstab(S, S.b, **k))):
        x, info = solve(maxit=0)
        assert info.status == G.MAXIT and info.iters == 0
        x, info = solve(maxit=1)
        x_o, o_info = osolve(maxit=1)
        assert info.status == o_info.status == G.MAXIT and info.iters == 1
        np.testing.assert_allclose(host(x), x_o, rtol=1e-12, atol=1e-14)
    # one unknown
    O = _dense(np.array([[3.0]]), [6.0])
    A, b = up(G, O)
    x, info = G.gmres(A, b, m=3, tol=1e-12)
    assert info.status == G.CONVERGED and host(x)[0] == pytest.approx(2.0, rel=1e-15)
    x, info = G.bicgstab(A, b, tol=1e-12)
    assert info.status == G.CONVERGED and host(x)[0] == pytest.approx(2.0, rel=1e-15)
    # nonzero initial guess
    S2, _, _ = oracle_scaled(problems.slabs_3d(12), 2)
    A, b = up(G, S2)
    x0 = torch.linspace(-1, 1, S2.n, dtype=torch.float64, device="cuda")
    x, info = G.gmres(A, b, x0, m=30, tol=1e-10)
    x_o, o_info = oracle.gmres(S2, S2.b, host(x0), m=30, tol=1e-10)
    _check_solver(info, o_info, host(x), x_o, 1e-10, 1e-8)
    x, info = G.bicgstab(A, b, x0, tol=1e-10)
    x_o, o_info = oracle.bicgstab(S2, S2.b, host(x0), tol=1e-10)
    _check_solver(info, o_info, host(x), x_o, 1e-10, 1e-8)


def test_solver_rejects_invalid_structure(G):
    Bad = problems.random_sparse(500, 4, 31)
    Bad.col_idx = Bad.col_idx.copy()
    Bad.col_idx[-1] = -2
    A, b = up(G, Bad)
    with pytest.raises(G.GskError) as e:
        G.bicgstab(A, b, tol=1e-8)
    assert e.value.code == G.ERR_INVALID_ARG
    with pytest.raises(G.GskError) as e:
        G.gmres(A, b, m=5, tol=1e-8)
    assert e.value.code == G.ERR_INVALID_ARG


def test_repeat_runs_are_bitwise_identical(G):
    import torch
    S, _, _ = oracle_scaled(problems.slabs_3d(18), 2)
    A, b = up(G, S)
    x1, i1 = G.bicgstab(A, b, tol=1e-10)
    x2, i2 = G.bicgstab(A, b, tol=1e-10)
    g1, j1 = G.gmres(A, b, m=30, tol=1e-10)
    g2, j2 = G.gmres(A, b, m=30, tol=1e-10)
    torch.cuda.synchronize()
    assert i1 == i2 and j1 == j2
    assert torch.equal(x1, x2) and torch.equal(g1, g2)


# ------------------------------------------------------------------ full benchmark size

@pytest.fixture(scope="module")
def slabs80():
    return problems.slabs_3d()


def _golden_slabs80():
    with open(os.path.join(HERE, "golden", "slabs80_oracle.json")) as f:
        return json.load(f)


def _sub_rows(P, rows):
    starts, ends = P.row_ptr[rows], P.row_ptr[rows + 1]
    counts = ends - starts
    rp = np.zeros(len(rows) + 1, np.int32)
    rp[1:] = np.cumsum(counts)
    sel = np.concatenate([np.arange(s, e) for s, e in zip(starts, ends)])
    return problems.Problem("sub", (len(rows),), rp, P.col_idx[sel].copy(), P.val[sel].copy(),
                            P.b[rows].copy()), sel


def test_slabs80_full_size_gs_and_spmv_sampled(G, slabs80):
    import torch
    P = slabs80
    A, b = up(G, P)
    rows = np.sort(np.random.default_rng(3).choice(P.n, size=4000, replace=False))
    rows = np.unique(np.concatenate([rows, [0, P.n - 1]]))
    sub, sel = _sub_rows(P, rows)
    for p in (1, 2):
        S, bs, nrm, w = G.gs_scale(A, b, p, want_weights=True)
        vo, bo, n_o, w_o = oracle.gs_scale(sub, sub.b, p)
        np.testing.assert_array_equal(host(S.val)[sel], vo)
        np.testing.assert_array_equal(host(bs)[rows], bo)
        np.testing.assert_array_equal(host(nrm)[rows], n_o)
        np.testing.assert_array_equal(host(w)[rows], w_o)
    x = np.random.default_rng(5).standard_normal(P.n)
    y = host(G.spmv(A, torch.from_numpy(x).cuda()))
    np.testing.assert_array_equal(y[rows], oracle.spmv(sub, x))
    St = G.stencil_from_csr(A, *P.dims)
    y = host(G.spmv(St, torch.from_numpy(x).cuda()))
    np.testing.assert_array_equal(y[rows], oracle.spmv(sub, x))


@pytest.mark.parametrize("operator", ["stencil", "csr"])
@pytest.mark.parametrize("key", ["gs2_bicgstab", "gs2_gmres30", "gs1_bicgstab", "gs1_gmres30"])
def test_slabs80_full_size_solves_match_oracle(G, slabs80, key, operator):
    """The bench's four solves at full size, in the bench's launch configuration (GS(p) out of
    place, then, for the stencil operator, packing of the scaled matrix)."""
    import torch
    gold = _golden_slabs80()
    run = gold["runs"][key]
    idx = np.array(gold["sample_idx"])
    p = 2 if key.startswith("gs2") else 1
    P = slabs80
    A, b = up(G, P)
    As, bs, _, w = G.gs_scale(A, b, p, want_weights=True)
    if operator == "stencil":
        As = G.stencil_from_csr(As, *P.dims)
    weights = None if p == 2 else w
    if key.endswith("bicgstab"):
        x, info = G.bicgstab(As, bs, tol=1e-10, stop_weights=weights)
    else:
        x, info = G.gmres(As, bs, m=30, tol=1e-10, stop_weights=weights)
    torch.cuda.synchronize()
    assert info.status == run["status"] == G.CONVERGED
    assert abs(info.iters - run["iters"]) <= max(1, 0.05 * run["iters"]), (info, run["iters"])
    assert info.relres_true < 1e-10
    xs = host(x)[idx]
    xo = np.array(run["x_sample"])
    assert np.linalg.norm(xs - xo) / np.linalg.norm(xo) <= 1e-8
    err = np.linalg.norm(host(x) - P.u_star) / np.linalg.norm(P.u_star)
    assert err == pytest.approx(run["err_vs_u_star"], rel=0.5, abs=1e-9)


@pytest.mark.parametrize("dims,conv,p", [((104, 104, 100), (30.0, -10.0, 5.0), 2),
                                         ((103, 101, 101), (30.0, -10.0, 5.0), 2),
                                         ((104, 104, 100), (10.0, 20.0, -5.0), 1),
                                         ((256, 4100), (25.0, 5.0), 2),
                                         ((300, 3500), (5.0, 1.0), 2),
                                         ((24, 20, 12), (30.0, -10.0, 5.0), 2)])
def test_bicgstab_stencil_equals_csr_bitwise(G, dims, conv, p):
    """Bi-CGSTAB on the packed stencil matrix returns the bits of the same solve on the CSR
    matrix (one tile per workgroup): x, counts, status, both residuals. From 2^20 rows the
    stencil solve's P and S run through the LDS window, two tiles per workgroup: rows in
    16-byte pairs where n and nx are even (the first, third and fourth cases), single rows
    otherwise (the second); x-lines wider than the window (the fifth) and small systems (the
    last) take the one-tile kernels. GS(1) runs with stop weights."""
    import torch
    P = problems.laplacian(dims, conv=conv)
    A, b = up(G, P)
    As, bs, _, w = G.gs_scale(A, b, p, want_weights=True)
    weights = None if p == 2 else w
    St = G.stencil_from_csr(As, *(list(P.dims) + [1] * (3 - len(P.dims))))
    xs, i_s = G.bicgstab(St, bs, tol=1e-10, stop_weights=weights)
    xc, i_c = G.bicgstab(As, bs, tol=1e-10, stop_weights=weights)
    torch.cuda.synchronize()
    assert i_s == i_c
    assert np.array_equal(host(xs), host(xc))


@pytest.mark.parametrize("dims", [(104, 104, 100), (103, 101, 101), (256, 4100)])
def test_gmres_large_stencil_equals_csr_bitwise(G, dims):
    """FP64 GMRES(30) on systems whose cycle working set exceeds the 256 MB last-level cache
    (over 10^6 rows): the stencil solve's Arnoldi product gathers through the LDS window
    (non-temporal basis and plane loads), the CSR solve through the LDS-staged CSR tiles. Two
    cycles (60 steps) return the same bits: x, counts, status, both residuals."""
    import torch
    P = problems.laplacian(dims, conv=(30.0, -10.0, 5.0)[:len(dims)])
    A, b = up(G, P)
    As, bs, _, _ = G.gs_scale(A, b, 2, want_weights=True)
    St = G.stencil_from_csr(As, *(list(P.dims) + [1] * (3 - len(P.dims))))
    xs, i_s = G.gmres(St, bs, m=30, tol=1e-12, maxit=60)
    xc, i_c = G.gmres(As, bs, m=30, tol=1e-12, maxit=60)
    torch.cuda.synchronize()
    assert i_s == i_c and i_s.iters == 60
    assert np.array_equal(host(xs), host(xc))
