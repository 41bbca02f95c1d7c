"""Serving with continuous batching: every result equals the same solve done alone.

Requests (a Bi-CGSTAB / GMRES(20) mix, GS(2) per request) arrive while others are on the GPU
and are admitted as the engine's rows and slots free up. Each Bi-CGSTAB result must equal
gsk_gs_scale + stencil packing + gsk_bicgstab on the same system alone, bit for bit (x, info);
each GMRES result, whether it ran on a lane or in a GMRES engine (FP64 or mixed precision),
must equal the single GMRES solve of that precision.
"""
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


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def pool(G, count=6, specs=None):
    out = []
    for sp in specs or problems.batch_specs(count, seed=21, n_min=8, n_max=28):
        P = problems.batch_system(sp)
        A = G.CsrMatrix.from_problem(P)
        d = list(P.dims) + [1] * (3 - len(P.dims))
        out.append({"A": A, "S": G.stencil_from_csr(A, *d), "b": dev(P.b), "grid": tuple(d),
                    "n": P.n})
    return out


def alone(G, s, method, mixed=False):
    As, bs, _, _ = G.gs_scale(s["A"], s["b"], 2, want_norms=False)
    M = G.stencil_from_csr(As, *s["grid"])
    if method == "gmres":
        return (G.gmres_mixed if mixed else G.gmres)(M, bs, m=20, tol=1e-8)
    return G.bicgstab(M, bs, tol=1e-8)


@pytest.mark.parametrize("realtime,mode,sizes", [(False, "lanes", "small"),
                                                 (True, "lanes", "small"),
                                                 (True, "engine", "small"),
                                                 (False, "engine-mixed", "small"),
                                                 (True, "engine-mixed", "workload")])
def test_serving_results_equal_solo(G, realtime, mode, sizes):
    """sizes "workload": six systems of the serving workload's own distribution (every 85th
    of the 512-system list: 32^3 twice, 53^3, 54^3, 76^3 and 64^2), arriving at 2,000
    requests/s, with GMRES in a mixed-precision engine, as the serving benchmark runs by
    default."""
    import torch
    from paper_0812_2769_amd import serve
    systems = pool(G, specs=problems.batch_specs(512)[::85][:6] if sizes == "workload" else None)
    rng = np.random.default_rng(3)
    n_req = 24
    rate = 2000.0 if sizes == "workload" else 400.0
    arrivals = np.cumsum(rng.exponential(1 / rate, size=n_req))
    picks = rng.integers(0, len(systems), size=n_req)
    kinds = rng.random(n_req) < 0.25
    reqs = [serve.Request(tag=k, arrival=float(arrivals[k]), A=systems[picks[k]]["S"],
                          b=systems[picks[k]]["b"], method="gmres" if kinds[k] else "bicgstab",
                          m=20, tol=1e-8, csr=systems[picks[k]]["A"],
                          grid=systems[picks[k]]["grid"]) for k in range(n_req)]
    # room for about two systems at a time: admission has to wait for retirements
    rows = sorted(((s["n"] + 255) // 256 * 256 for s in systems), reverse=True)
    mixed = mode == "engine-mixed"
    srv = serve.Server(rows[0] + rows[1], 4, check_every=8, graph=True,
                       gmres_rows=max(s["n"] for s in systems), m_max=20,
                       gmres_mode="lanes" if mode == "lanes" else "engine",
                       gmres_precision="mixed" if mixed else "fp64",
                       gmres_engine_rows=2 * (rows[0] + rows[1]), gmres_engine_systems=4)
    done = srv.serve(reqs, realtime=realtime)
    srv.close()
    assert sorted(d.tag for d in done) == list(range(n_req))
    # admissions were spread over the run (requests joined while others were on the GPU)
    assert len({round(d.admitted, 6) for d in done if d.method == "bicgstab"}) > 1
    torch.cuda.synchronize()
    ref = {}
    for d in done:
        key = (int(picks[d.tag]), d.method)
        if key not in ref:
            x, info = alone(G, systems[key[0]], key[1], mixed)
            ref[key] = (x.cpu().numpy(), info)
        xr, ir = ref[key]
        assert d.info == ir, (d.tag, d.method, d.info, ir)
        assert np.array_equal(d.x.cpu().numpy(), xr), (d.tag, d.method)


def test_request_larger_than_engine_is_an_error(G):
    from paper_0812_2769_amd import serve
    systems = pool(G, count=2)
    big = max(systems, key=lambda s: s["n"])
    reqs = [serve.Request(tag=0, arrival=0.0, A=big["S"], b=big["b"], method="bicgstab",
                          tol=1e-8, csr=big["A"], grid=big["grid"])]
    srv = serve.Server(256, 2, graph=False)
    with pytest.raises(ValueError):
        srv.serve(reqs, realtime=False)
    srv.close()


def test_served_results_match_the_oracle(G):
    """Served results checked against the oracle itself (GS(2), then Bi-CGSTAB or
    GMRES(20), tol 1e-8): equal status, the true residual below tol, iteration counts within
    max(2, 10%) (rounding moves them), and x within the conditioning bound of the oracle's
    x. The engines are sized from the device's free memory (no row counts given). GMRES(20)
    requests use the systems on which the oracle needs at most 10 cycles: over tens of
    restarts (27 on system 0) the step count of restarted GMRES moves by more than 10% with
    rounding alone, which the GMRES parity tests cover with their own bars."""
    import torch
    import oracle
    from paper_0812_2769_amd import serve
    specs = problems.batch_specs(8, seed=31, n_min=8, n_max=16)
    systems = pool(G, specs=specs)
    hosts = [problems.batch_system(sp) for sp in specs]
    n_req = 16
    few_cycles = [2, 4, 7]       # the oracle's GMRES(20) converges in <= 10 cycles on these
    pick = list(range(8)) + [few_cycles[k % 3] for k in range(8)]
    reqs = [serve.Request(tag=k, arrival=0.001 * k, A=systems[pick[k]]["S"],
                          b=systems[pick[k]]["b"], method="gmres" if k >= 8 else "bicgstab",
                          m=20, tol=1e-8, csr=systems[pick[k]]["A"], grid=systems[pick[k]]["grid"])
            for k in range(n_req)]
    srv = serve.Server(0, 8, graph=True, m_max=20, gmres_mode="engine",
                       gmres_precision="fp64", gmres_engine_systems=8)
    assert srv.sizing["bicgstab_rows"] >= 256 and srv.sizing["gmres_rows"] >= 256
    done = srv.serve(reqs, realtime=True)
    srv.close()
    torch.cuda.synchronize()
    assert sorted(d.tag for d in done) == list(range(n_req))
    for d in done:
        P = hosts[pick[d.tag]]
        vo, bo, _, _ = oracle.gs_scale(P, P.b, 2)
        S = P.copy()
        S.val, S.b = vo, bo
        if d.method == "gmres":
            xo, io = oracle.gmres(S, bo, m=20, tol=1e-8)
        else:
            xo, io = oracle.bicgstab(S, bo, tol=1e-8)
        assert d.info.status == io.status, (d.tag, d.info, io)
        assert abs(d.info.iters - io.iters) <= max(2, 0.1 * io.iters), (d.tag, d.info, io)
        if io.status == oracle.CONVERGED:
            assert d.info.relres_true < 1e-8
            A = S.dense()
            x = d.x.cpu().numpy()
            bound = 10 * np.linalg.cond(A) * 1e-8
            assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= bound, (d.tag, bound)
