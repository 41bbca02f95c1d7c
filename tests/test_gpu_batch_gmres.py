"""GMRES(m) engines (FP64 and mixed precision) through the C ABI.

Each system in a GMRES engine runs the single solver's workgroup bodies on its own rows and
reduces its own partials in the single solver's order, so the bar is bit-for-bit equality
with gsk_gmres (FP64 engine) or gsk_gmres_mixed (mixed engine): x, step and restart counts,
status and both residuals. That must hold with admissions between chunks, under graph
replay, with the GS(p) stage inside the engine, for stencil and CSR systems. One mixed system
is also compared with the oracle's mixed-precision GMRES directly.
"""
import numpy as np
import pytest

import oracle
from paper_0812_2769_amd import problems

pytestmark = pytest.mark.gpu

M = 20
MAXIT = 600     # restarted GMRES(20) stagnates on some jump problems: bound the runs


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


def scaled(G, P, p=2, stencil=True):
    A = G.CsrMatrix.from_problem(P)
    As, bs, _, w = G.gs_scale(A, dev(P.b), p, want_weights=(p != 2))
    Ms = G.stencil_from_csr(As, *grid_of(P)) if stencil else As
    return Ms, bs, (w if p != 2 else None)


def systems(G):
    """3D and 2D stencils, a CSR system, GS(1) with stop weights, ragged and tiny sizes."""
    specs = problems.batch_specs(5, seed=17, n_min=6, n_max=18)
    out = []
    for i, sp in enumerate(specs):
        P = problems.batch_system(sp)
        out.append(scaled(G, P, p=1 if i == 2 else 2, stencil=(i != 3)))
    out.append(scaled(G, problems.laplacian((13, 11, 7), conv=(40.0, -25.0, 10.0))))
    out.append(scaled(G, problems.laplacian((3, 2)), stencil=False))
    return out


def solo(G, syst, mixed, tol):
    f = G.gmres_mixed if mixed else G.gmres
    res = []
    for A, b, w in syst:
        x, info = f(A, b, m=M, tol=tol, stop_weights=w, maxit=MAXIT)
        res.append((host(x), info))
    return res


def same(a, b, what):
    (xa, ia), (xb, ib) = a, b
    assert ia == ib, (what, ia, ib)
    assert np.array_equal(xa, xb), what


def run_engine(G, eng, syst, tol, gs=None):
    import torch
    xs = [torch.zeros_like(b) for _, b, _ in syst]
    pending = list(range(len(syst)))
    results, chunks, late = {}, 0, False
    while len(results) < len(syst):
        while pending:
            k = pending[0]
            A, b, w = syst[k]
            ok = (eng.submit_gs(A, b, xs[k], p=gs[k], tol=tol, tag=k, maxit=MAXIT) if gs else
                  eng.submit(A, b, xs[k], tol=tol, tag=k, stop_weights=w, maxit=MAXIT))
            if not ok:
                break
            late = late or chunks > 0
            pending.pop(0)
        eng.run(1)
        chunks += 1
        for tag, info in eng.poll(wait=True):
            results[tag] = info
        assert chunks < 3000
    torch.cuda.synchronize()
    return xs, results, late


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gmres_engine_equals_solo(G, precision, graph):
    syst = systems(G)
    tol = 1e-10
    ref = solo(G, syst, precision == "mixed", tol)
    assert sum(i.status == G.CONVERGED for _, i in ref) >= len(ref) // 2
    rows = sorted(((A.n + 511) // 512 * 512 for A, _, _ in syst), reverse=True)
    eng = G.Engine(rows[0] + rows[1], 3, graph=graph, method="gmres", m=M,
                   precision=precision)
    xs, res, late = run_engine(G, eng, syst, tol)
    assert late   # some systems were admitted while others ran
    for k in range(len(syst)):
        same((host(xs[k]), res[k]), ref[k], (precision, k))
    u = eng.usage()
    assert u["active"] == 0 and u["free_rows"] == u["max_rows"] // 256 * 256
    eng.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gmres_engine_gs_stage_equals_solo(G, precision):
    import torch
    specs = problems.batch_specs(4, seed=23, n_min=8, n_max=20)
    mixed = precision == "mixed"
    f = G.gmres_mixed if mixed else G.gmres
    eng = G.Engine(1 << 17, 8, graph=True, method="gmres", m=M, precision=precision)
    ref, syst, ps = {}, [], []
    for i, sp in enumerate(specs):
        P = problems.batch_system(sp)
        p = 1 if i == 1 else 2
        stencil = i != 2
        Ms, bs, w = scaled(G, P, p, stencil)
        x, info = f(Ms, bs, m=M, tol=1e-10, stop_weights=w, maxit=MAXIT)
        ref[i] = (host(x), info)
        A = G.CsrMatrix.from_problem(P)
        syst.append((G.stencil_from_csr(A, *grid_of(P)) if stencil else A, dev(P.b), None))
        ps.append(p)
    xs, res, _ = run_engine(G, eng, syst, 1e-10, gs=ps)
    for i in ref:
        same((host(xs[i]), res[i]), ref[i], (precision, i))
    eng.close()


def test_mixed_engine_matches_oracle(G):
    P = problems.batch_system(problems.batch_specs(1, seed=29, n_min=14, n_max=14)[0])
    vo, bo, _, _ = oracle.gs_scale(P, P.b, 2)
    S = P.copy()
    S.val, S.b = vo, bo
    xo, io = oracle.gmres_ir(S, bo, m=M, tol=1e-10)
    Ms, bs, _ = scaled(G, P)
    eng = G.Engine(1 << 14, 2, method="gmres", m=M, precision="mixed")
    xs, res, _ = run_engine(G, eng, [(Ms, bs, None)], 1e-10)
    assert res[0].status == io.status == G.CONVERGED
    assert abs(res[0].iters - io.iters) <= max(M, 0.05 * io.iters)
    assert np.linalg.norm(host(xs[0]) - xo) / np.linalg.norm(xo) <= 1e-8
    eng.close()


@pytest.mark.parametrize("precision,rows", [("fp64", 13 << 20), ("mixed", 27 << 20)])
def test_gmres_engine_basis_beyond_2gib(G, precision, rows):
    """An engine whose basis (m+1 columns over its whole row space) exceeds 2^31 bytes reads it
    with 64-bit addresses; a few small systems in it still return the single solves' bits."""
    width = 8 if precision == "fp64" else 4
    assert (M + 1) * width * rows >= 2 ** 31
    syst = systems(G)[:4]
    tol = 1e-10
    ref = solo(G, syst, precision == "mixed", tol)
    eng = G.Engine(rows, 4, graph=True, method="gmres", m=M, precision=precision)
    xs, res, _ = run_engine(G, eng, syst, tol)
    for k in range(len(syst)):
        same((host(xs[k]), res[k]), ref[k], (precision, k))
    eng.close()


def test_gmres_engine_rejects_bad_systems(G):
    import torch
    P = problems.laplacian((8, 8))
    rp = P.row_ptr.copy()
    rp[5] = rp[6] + 1        # not monotone
    bad = G.CsrMatrix.from_numpy(rp, P.col_idx, P.val)
    val = P.val.copy()
    val[P.row_ptr[7]:P.row_ptr[8]] = 0.0      # row 7 all zero
    zero_row = G.CsrMatrix.from_numpy(P.row_ptr, P.col_idx, val)
    good, bg, _ = scaled(G, P)
    for precision in ("fp64", "mixed"):
        eng = G.Engine(4096, 4, method="gmres", m=M, precision=precision)
        xb = torch.zeros(P.n, dtype=torch.float64, device="cuda")
        xz = torch.zeros_like(xb)
        xg = torch.zeros_like(bg)
        assert eng.submit(bad, dev(P.b), xb, tol=1e-8, tag=0)
        assert eng.submit_gs(zero_row, dev(P.b), xz, p=2, tol=1e-8, tag=1)
        assert eng.submit(good, bg, xg, tol=1e-8, tag=2)
        done = {}
        for _ in range(200):
            eng.run(1)
            done.update(dict(eng.poll()))
            if len(done) == 3:
                break
        assert done[0].status == -1 and done[1].status == -2, (precision, done)
        assert done[2].status == G.CONVERGED
        assert not xb.any() and not xz.any()
        eng.close()


def test_gmres_engine_arguments(G):
    with pytest.raises(G.GskError):
        G.Engine(1024, 4, method="gmres", m=0)
    with pytest.raises(G.GskError):
        G.Engine(1024, 4, method="gmres", m=G.MAX_RESTART + 1 if hasattr(G, "MAX_RESTART")
                 else 65)
    with pytest.raises(G.GskError):
        G.Engine(1024, 4, method="bicgstab", precision="mixed", inner_reduction=1.5)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gmres_engine_streaming_largest_systems_equal_solo(G, precision):
    """The 14 largest 3D systems of the 512-system workload (about 11 M rows: the engine's
    admitted cycle working set is far beyond the 256 MB last-level cache, so its chunks take
    the non-temporal load policy and, in FP64, the LDS-window product), each bounded to five
    GMRES(20) cycles. Alone, each system's cycle fits in the cache and the single solver takes
    ordinary loads and the plain product. The results must still be equal bit for bit."""
    import torch
    specs = problems.batch_specs(512)
    sizes = [int(np.prod(s["dims"])) for s in specs]
    pick = sorted((i for i, s in enumerate(specs) if len(s["dims"]) == 3),
                  key=sizes.__getitem__)[-14:]
    width = 4 if precision == "mixed" else 8
    assert (M + 2) * width * sum(sizes[i] for i in pick) > 2 * 256 * 2 ** 20
    syst = [scaled(G, problems.batch_system(specs[i])) for i in pick]
    f = G.gmres_mixed if precision == "mixed" else G.gmres
    ref = [(host(x), info) for x, info in
           (f(A, b, m=M, tol=1e-8, maxit=5 * M) for A, b, _ in syst)]
    rows = sum((A.n + 511) // 512 * 512 for A, _, _ in syst)
    eng = G.Engine(rows, len(syst), graph=True, method="gmres", m=M, precision=precision)
    xs = [torch.zeros_like(b) for _, b, _ in syst]
    for k, (A, b, _) in enumerate(syst):
        assert eng.submit(A, b, xs[k], tol=1e-8, tag=k, maxit=5 * M)
    res = {}
    for _ in range(100):
        eng.run(1)
        res.update(dict(eng.poll(wait=True)))
        if len(res) == len(syst):
            break
    torch.cuda.synchronize()
    eng.close()
    assert len(res) == len(syst)
    for k in range(len(syst)):
        same((host(xs[k]), res[k]), ref[k], (precision, pick[k]))
