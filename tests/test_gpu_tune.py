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


def solve(G, systems, k, units=0):
    import torch
    rows = sum((s["n"] + 511) // 512 * 512 for s in systems)
    eng = G.Engine(rows, len(systems), check_every=k, graph=True, tile_units=units)
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
