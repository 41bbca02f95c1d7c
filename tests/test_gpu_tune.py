"""The engine's launch shape (tiles per workgroup) and chunk length are pure scheduling choices:
every choice gives the same bits, so the measured choice (paper_0812_2769_amd.tune) can only
change the time, never the result."""
import numpy as np
import pytest

from paper_0812_2769_amd import problems

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0812_2769_amd import gsk
    return gsk


def batch(G, count=6):
    import torch
    out = []
    for sp in problems.batch_specs(count, seed=31, n_min=8, n_max=24):
        P = problems.batch_system(sp)
        A = G.CsrMatrix.from_problem(P)
        d = list(P.dims) + [1] * (3 - len(P.dims))
        out.append({"S": G.stencil_from_csr(A, *d), "b": torch.from_numpy(P.b).cuda(),
                    "n": P.n})
    return out


def solve(G, systems, k, units=0, class_shapes=None):
    import torch
    rows = sum((s["n"] + 511) // 512 * 512 for s in systems)
    eng = G.Engine(rows, len(systems), check_every=k, graph=True, tile_units=units,
                   class_shapes=class_shapes)
    xs = [torch.zeros_like(s["b"]) for s in systems]
    for i, s in enumerate(systems):
        assert eng.submit_gs(s["S"], s["b"], xs[i], p=2, tol=1e-10, tag=i)
    res = {}
    while len(res) < len(systems):
        eng.run(1)
        res.update(dict(eng.poll(wait=True)))
    torch.cuda.synchronize()
    eng.close()
    return [x.cpu().numpy() for x in xs], res


def test_chunk_length_does_not_change_results(G):
    systems = batch(G)
    x4, r4 = solve(G, systems, 4)
    x16, r16 = solve(G, systems, 16)
    assert r4 == r16
    for a, b in zip(x4, x16):
        assert np.array_equal(a, b)


def test_tuner_picks_a_candidate(G):
    from paper_0812_2769_amd import tune
    systems = batch(G, 4)
    t = tune.tune_check_every(systems, candidates=(4, 8), maxit=20)
    assert t["best"] in (4, 8) and set(t["seconds"]) == {4, 8}
    assert all(v > 0 for v in t["seconds"].values())
    with pytest.raises(ValueError):
        tune.tune_check_every(systems, candidates=(3,), maxit=4)


def test_tile_shape_does_not_change_results(G):
    import torch
    systems = batch(G, 8)
    # a CSR system too (two tiles through LDS one after the other)
    P = problems.laplacian((30, 27), conv=(20.0, 5.0))
    A = G.CsrMatrix.from_problem(P)
    systems.append({"S": A, "b": torch.from_numpy(P.b).cuda(), "n": P.n})
    x1, r1 = solve(G, systems, 8, units=1)
    x2, r2 = solve(G, systems, 8, units=2)
    assert r1 == r2
    for a, b in zip(x1, x2):
        assert np.array_equal(a, b)


def test_engine_tuner_covers_shapes(G):
    from paper_0812_2769_amd import tune
    systems = batch(G, 4)
    t = tune.tune_engine(systems, shapes=(1, 2), chunks=(8,), maxit=16)
    assert t["best"] in ((1, 8), (2, 8)) and set(t["seconds"]) == {(1, 8), (2, 8)}
    with pytest.raises(G.GskError):
        G.Engine(1024, 2, method="gmres", tile_units=2)


def test_class_shapes_do_not_change_results(G):
    """Per-size-class launch shapes (each class its own launches, rows in pairs of tiles) give
    the bits of the one-shape engine, for every shape in every class: small 2D and 3D
    stencils, a CSR matrix, a 3D stencil above the large-class bound, ragged sizes."""
    import torch
    systems = batch(G, 8)
    P = problems.laplacian((30, 27), conv=(20.0, 5.0))
    systems.append({"S": G.CsrMatrix.from_problem(P), "b": torch.from_numpy(P.b).cuda(),
                    "n": P.n})
    P = problems.laplacian((66, 64, 63), conv=(10.0, -5.0, 3.0))
    assert P.n >= G.CLASS_LARGE_ROWS
    A = G.CsrMatrix.from_problem(P)
    systems.append({"S": G.stencil_from_csr(A, 66, 64, 63), "b": torch.from_numpy(P.b).cuda(),
                    "n": P.n})
    classes = {G.size_class(s["S"]) for s in systems}
    assert classes == set(G.SIZE_CLASSES)
    x0, r0 = solve(G, systems, 8, units=1)
    for shapes in ({"2d": "tile", "3d_small": "pair_tile_u", "3d_large": "pair"},
                   {"2d": "pair", "3d_small": "tile", "3d_large": "pair_tile_u"},
                   {"3d_large": "tile"}):
        x, r = solve(G, systems, 8, class_shapes=shapes)
        assert r == r0, shapes
        for a, b in zip(x0, x):
            assert np.array_equal(a, b), shapes


def test_class_shapes_argument_checks(G):
    with pytest.raises(G.GskError):
        G.Engine(1024, 2, method="gmres", class_shapes={"2d": "pair"})
    with pytest.raises(G.GskError):
        G.Engine(1024, 2, precision="mixed", class_shapes={"2d": "pair"})
    with pytest.raises(G.GskError):
        G.Engine(1024, 2, class_shapes={"2d": 4})
