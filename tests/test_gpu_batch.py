"""Batched Bi-CGSTAB and the continuous-batching engine through the C ABI.

Each system in a batch is solved exactly as gsk_bicgstab solves it alone (same operations,
same per-tile partial sums in the same order), so the bar is bit-for-bit equality with the
single solve: x, iteration counts, statuses and residuals. That holds in one batch, when
systems are admitted while others run (the engine), and when every chunk is a replay of a
captured HIP graph. The single solver itself is checked against the oracle elsewhere; one
batch system is also compared with the oracle here directly.
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


def scaled(G, P, p=2, stencil=True):
    A = G.CsrMatrix.from_problem(P)
    As, bs, _, w = G.gs_scale(A, dev(P.b), p, want_weights=(p != 2))
    M = G.stencil_from_csr(As, *grid_of(P)) if stencil else As
    return M, bs, (w if p != 2 else None)


def systems(G):
    """A mix of kinds and sizes: 3D and 2D stencils, a CSR system, GS(1) with stop weights,
    ragged row counts, a tiny system."""
    specs = problems.batch_specs(6, seed=7, n_min=6, n_max=20)
    out = []
    for i, sp in enumerate(specs):
        P = problems.batch_system(sp)
        out.append(scaled(G, P, p=1 if i == 2 else 2, stencil=(i != 3)))
    out.append(scaled(G, problems.laplacian((13, 11, 7), conv=(40.0, -25.0, 10.0))))
    out.append(scaled(G, problems.laplacian((3, 2)), stencil=False))
    # even row count and x-line (two rows per thread in two-tile units), and an x-line wider
    # than the two-tile units' LDS window (global gathers)
    out.append(scaled(G, problems.laplacian((12, 10, 6), conv=(5.0, 7.0, -3.0))))
    out.append(scaled(G, problems.laplacian((300, 3), conv=(2.0, 1.0))))
    return out


def solo(G, syst, tol=1e-10):
    res = []
    for M, b, w in syst:
        x, info = G.bicgstab(M, b, tol=tol, stop_weights=w)
        res.append((host(x), info))
    return res


def same(a, b):
    (xa, ia), (xb, ib) = a, b
    assert ia == ib, (ia, ib)
    assert np.array_equal(xa, xb)


def test_batch_equals_solo(G):
    syst = systems(G)
    ref = solo(G, syst)
    assert all(i.status == G.CONVERGED for _, i in ref)
    # bicgstab_batch takes one tol and no per-system weights: compare the unweighted ones
    idx = [k for k, (_, _, w) in enumerate(syst) if w is None]
    xs, infos = G.bicgstab_batch([syst[k][0] for k in idx], [syst[k][1] for k in idx],
                                 tol=1e-10)
    for j, k in enumerate(idx):
        same((host(xs[j]), infos[j]), ref[k])


@pytest.mark.parametrize("graph,tile_units,shapes", [
    (False, 1, None), (True, 1, None), (False, 2, None), (True, 2, None),
    (True, 0, {"2d": "tile", "3d_small": "pair", "3d_large": "pair_tile_u"}),
    (False, 0, {"2d": "pair_tile_u", "3d_small": "tile"})])
def test_engine_continuous_admission_equals_solo(G, graph, tile_units, shapes):
    """Systems admitted while others run (room for part of the set), with one shape or per-class
    shapes (per-class unit lists rebuilt at every admission and retirement), eager or replayed
    from graphs: every result equals the single solve bit for bit."""
    import torch
    syst = systems(G)
    ref = solo(G, syst)
    # room for only part of the set at a time: later systems wait for rows and slots
    unit = 512 if shapes else 256 * tile_units
    rows = sorted(((M.n + unit - 1) // unit * unit for M, _, _ in syst), reverse=True)
    eng = G.Engine(max_rows=rows[0] + rows[1], max_systems=3, check_every=8, graph=graph,
                   tile_units=tile_units, class_shapes=shapes)
    xs = [torch.zeros_like(b) for _, b, _ in syst]
    pending = list(range(len(syst)))
    results = {}
    admitted_late = False
    chunks = 0
    while len(results) < len(syst):
        while pending:
            k = pending[0]
            M, b, w = syst[k]
            if not eng.submit(M, b, xs[k], tol=1e-10, tag=k, stop_weights=w):
                break
            admitted_late = admitted_late or chunks > 0
            pending.pop(0)
        eng.run(1)
        chunks += 1
        for tag, info in eng.poll(wait=True):
            results[tag] = info
        assert chunks < 5000
    assert admitted_late   # some systems joined while others were running
    torch.cuda.synchronize()
    for k in range(len(syst)):
        same((host(xs[k]), results[k]), ref[k])
    u = eng.usage()
    assert u["active"] == 0 and u["free_rows"] == u["max_rows"] // 256 * 256
    eng.close()


def test_engine_full_and_usage(G):
    import torch
    P = problems.laplacian((20, 20))
    M, b, _ = scaled(G, P)
    eng = G.Engine(max_rows=512, max_systems=4)
    x1, x2 = torch.zeros_like(b), torch.zeros_like(b)
    assert eng.submit(M, b, x1, tol=1e-8, tag=1)          # 400 rows -> 2 tiles of 256
    assert not eng.submit(M, b, x2, tol=1e-8, tag=2)      # no rows left
    u = eng.usage()
    assert u["active"] == 1 and u["free_rows"] == 0
    done = {}
    for _ in range(200):
        eng.run(1)
        done.update(dict(eng.poll()))
        if 1 in done:
            break
    assert done[1].status == G.CONVERGED
    assert eng.submit(M, b, x2, tol=1e-8, tag=2)          # rows were freed
    eng.close()


def test_engine_invalid_csr_system_reported(G):
    import torch
    P = problems.laplacian((8, 8))
    rp = P.row_ptr.copy()
    rp[5] = rp[6] + 1        # not monotone
    bad = G.CsrMatrix.from_numpy(rp, P.col_idx, P.val)
    good, bg, _ = scaled(G, P)
    eng = G.Engine(max_rows=1024, max_systems=4)
    xb, xg = torch.zeros(P.n, dtype=torch.float64, device="cuda"), torch.zeros_like(bg)
    assert eng.submit(bad, dev(P.b), xb, tol=1e-8, tag=0)
    assert eng.submit(good, bg, xg, tol=1e-8, tag=1)
    done = {}
    for _ in range(200):
        eng.run(1)
        done.update(dict(eng.poll()))
        if len(done) == 2:
            break
    assert done[0].status < 0
    assert done[1].status == G.CONVERGED
    assert not xb.any()      # an invalid system's x is left alone
    eng.close()


def test_batch_system_matches_oracle(G):
    P = problems.batch_system(problems.batch_specs(1, seed=11, n_min=14, n_max=14)[0])
    vo, bo, _, _ = oracle.gs_scale(P, P.b, 2)
    S = P.copy()
    S.val, S.b = vo, bo
    xo, io = oracle.bicgstab(S, bo, tol=1e-10)
    M, b, _ = scaled(G, P)
    xs, infos = G.bicgstab_batch([M], [b], tol=1e-10)
    assert infos[0].status == io.status == G.CONVERGED
    assert abs(infos[0].iters - io.iters) <= max(1, 0.05 * io.iters)
    assert np.max(np.abs(host(xs[0]) - xo)) <= 1e-8 * np.max(np.abs(xo))


def test_engine_argument_errors(G):
    with pytest.raises(G.GskError):
        G.Engine(max_rows=0, max_systems=4)
    with pytest.raises(G.GskError):
        G.Engine(max_rows=1024, max_systems=4, check_every=7, graph=True)


@pytest.mark.parametrize("graph,tile_units", [(False, 1), (True, 1), (True, 2)])
def test_engine_gs_stage_equals_solo(G, graph, tile_units):
    """GS(p) inside the engine (first chunk) + Bi-CGSTAB == gsk_gs_scale (+ stencil packing)
    + gsk_bicgstab, bit for bit, for stencil and CSR systems, p = 2 and p = 1."""
    import torch
    specs = problems.batch_specs(5, seed=9, n_min=8, n_max=24)
    eng = G.Engine(max_rows=1 << 17, max_systems=8, graph=graph, tile_units=tile_units)
    ref, xs = {}, {}
    for i, sp in enumerate(specs):
        P = problems.batch_system(sp)
        p = 1 if i == 1 else 2
        stencil = i != 2
        A = G.CsrMatrix.from_problem(P)
        b = dev(P.b)
        As, bs, _, w = G.gs_scale(A, b, p, want_weights=(p != 2))
        Ms = G.stencil_from_csr(As, *grid_of(P)) if stencil else As
        x, info = G.bicgstab(Ms, bs, tol=1e-10, stop_weights=w if p != 2 else None)
        ref[i] = (host(x), info)
        M = G.stencil_from_csr(A, *grid_of(P)) if stencil else A
        xs[i] = torch.zeros_like(b)
        assert eng.submit_gs(M, b, xs[i], p=p, tol=1e-10, tag=i)
    done = {}
    for _ in range(2000):
        eng.run(1)
        done.update(dict(eng.poll()))
        if len(done) == len(specs):
            break
    torch.cuda.synchronize()
    for i in ref:
        same((host(xs[i]), done[i]), ref[i])
    eng.close()


def test_engine_gs_stage_zero_row(G):
    import torch
    P = problems.laplacian((6, 6))
    val = P.val.copy()
    val[P.row_ptr[7]:P.row_ptr[8]] = 0.0      # row 7 all zero
    A = G.CsrMatrix.from_numpy(P.row_ptr, P.col_idx, val)
    eng = G.Engine(max_rows=256, max_systems=2)
    x = torch.zeros(P.n, dtype=torch.float64, device="cuda")
    assert eng.submit_gs(A, dev(P.b), x, p=2, tol=1e-8, tag=5)
    eng.run(1)
    done = dict(eng.poll())
    assert done[5].status == -2 and not x.any()
    eng.close()


@pytest.mark.parametrize("tile_units", [1, 2])
def test_batch512_real_sizes_equal_solo(G, tile_units):
    """Systems of the 512-system batch workload at their own sizes: every 32nd of the seeded
    list plus its largest 3D (96^3) and 2D systems, 1.78 M rows in all. They run as the
    benchmark runs them: GS(2) inside the engine, chunks of 8 iterations replayed from a HIP
    graph, tol 1e-8, one or two tiles per workgroup. Each result must equal bit for bit what
    gsk_gs_scale, stencil packing and gsk_bicgstab give for that system alone."""
    import torch
    specs = problems.batch_specs(512)
    sizes = [int(np.prod(s["dims"])) for s in specs]
    largest = [max((i for i, s in enumerate(specs) if len(s["dims"]) == d),
                   key=sizes.__getitem__) for d in (2, 3)]
    pick = sorted(set(range(0, 512, 32)) | set(largest))
    assert sizes[largest[1]] == 96 ** 3
    unit = 256 * tile_units
    built = []
    for i in pick:
        P = problems.batch_system(specs[i])
        built.append((P, G.CsrMatrix.from_problem(P), dev(P.b)))
    rows = sum(-(-P.n // unit) * unit for P, _, _ in built)
    eng = G.Engine(max_rows=rows, max_systems=len(built), check_every=8, graph=True,
                   tile_units=tile_units)
    ref, xs = {}, {}
    for k, (P, A, b) in enumerate(built):
        As, bs, _, _ = G.gs_scale(A, b, 2)
        x, info = G.bicgstab(G.stencil_from_csr(As, *grid_of(P)), bs, tol=1e-8)
        ref[k] = (host(x), info)
        xs[k] = torch.zeros_like(b)
        assert eng.submit_gs(G.stencil_from_csr(A, *grid_of(P)), b, xs[k], p=2, tol=1e-8,
                             tag=k)
    done = {}
    for _ in range(5000):
        eng.run(1)
        done.update(dict(eng.poll()))
        if len(done) == len(built):
            break
    torch.cuda.synchronize()
    assert len(done) == len(built)
    for k in ref:
        same((host(xs[k]), done[k]), ref[k])
    eng.close()


def test_engine_beyond_the_cache_equals_solo(G):
    """The 14 largest 3D systems of the 512-system workload (about 11 M rows, over 600 MB of
    engine vectors: far beyond the 256 MB last-level cache) in one engine with per-class
    launch shapes, as the benchmark runs them. Each result must equal bit for bit what the
    single solver gives for that system alone."""
    import torch
    specs = problems.batch_specs(512)
    sizes = [int(np.prod(s["dims"])) for s in specs]
    pick = sorted((i for i, s in enumerate(specs) if len(s["dims"]) == 3),
                  key=sizes.__getitem__)[-14:]
    rows = sum(-(-sizes[i] // 512) * 512 for i in pick)
    assert 7 * 8 * rows > 2 * 256 * 2 ** 20
    eng = G.Engine(max_rows=rows, max_systems=len(pick), check_every=16, graph=True,
                   class_shapes={"2d": "pair", "3d_small": "pair_tile_u",
                                 "3d_large": "pair_tile_u"})
    ref, xs, keep = {}, {}, []
    for k, i in enumerate(pick):
        P = problems.batch_system(specs[i])
        A, b = G.CsrMatrix.from_problem(P), dev(P.b)
        As, bs, _, _ = G.gs_scale(A, b, 2)
        x, info = G.bicgstab(G.stencil_from_csr(As, *grid_of(P)), bs, tol=1e-8)
        ref[k] = (host(x), info)
        del As, bs, x
        xs[k] = torch.zeros_like(b)
        S = G.stencil_from_csr(A, *grid_of(P))
        keep.append((S, b))
        assert eng.submit_gs(S, b, xs[k], p=2, tol=1e-8, tag=k)
    done = {}
    for _ in range(5000):
        eng.run(1)
        done.update(dict(eng.poll()))
        if len(done) == len(pick):
            break
    torch.cuda.synchronize()
    assert len(done) == len(pick)
    for k in ref:
        same((host(xs[k]), done[k]), ref[k])
    eng.close()


def test_large_single_solves_equal_engine_on_every_exit(G):
    """A single solve of a system of over 2,048 tiles splits its finalize sums over four
    workgroups; the engine sums each system's partials in one. The results must still be equal
    bit for bit, whatever ends the solve: the iteration cap, loose tolerances (half- or
    full-step exits), a converged solve, GS(1) with stop weights, the stencil product (LDS
    window) and the CSR product."""
    import torch
    P = problems.laplacian((84, 84, 84), conv=(30.0, -20.0, 10.0))
    assert P.n > 2048 * 256
    cases = []
    for stencil in (True, False):
        M, b, _ = scaled(G, P, 2, stencil)
        for tol, maxit in ((1e-8, 3), (0.9, None), (0.3, None), (1e-6, None)):
            cases.append((M, b, None, tol, maxit))
    M, b, w = scaled(G, P, 1, True)
    cases.append((M, b, w, 1e-6, None))
    ref = []
    for M, b, w, tol, maxit in cases:
        x, info = G.bicgstab(M, b, tol=tol, maxit=maxit, stop_weights=w)
        ref.append((host(x), info))
    assert any(i.status == G.MAXIT for _, i in ref)
    assert any(i.status == G.CONVERGED and i.iters > 10 for _, i in ref)
    unit = 256
    rows = sum((M.n + unit - 1) // unit * unit for M, _, _, _, _ in cases)
    eng = G.Engine(max_rows=rows, max_systems=len(cases), check_every=8, graph=True)
    xs = [torch.zeros_like(b) for _, b, _, _, _ in cases]
    for k, (M, b, w, tol, maxit) in enumerate(cases):
        assert eng.submit(M, b, xs[k], tol=tol, tag=k, maxit=maxit, stop_weights=w)
    done = {}
    for _ in range(5000):
        eng.run(1)
        done.update(dict(eng.poll()))
        if len(done) == len(cases):
            break
    torch.cuda.synchronize()
    assert len(done) == len(cases)
    for k in range(len(cases)):
        same((host(xs[k]), done[k]), ref[k])
    eng.close()
