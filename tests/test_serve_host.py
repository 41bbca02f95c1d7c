"""The serving loop's scheduling on the CPU, with a stand-in engine backed by the oracle.

The stand-in admits a system while it has rows (whole 256-row tiles) and a slot free, solves
it with the oracle (GS(2), then Bi-CGSTAB or GMRES(m)), and reports it done after as many
chunks as its iteration count needs, so that systems of different lengths overlap and retire
out of order. The tests check the scheduler: every request is served exactly once, with the
result of its solve alone; requests are never admitted before they arrive; admission by free
device memory (a stand-in memory probe that counts what the admitted requests hold) defers
requests until retirements free memory; a request that does not fit is overtaken by later
ones that do, until it has waited max_skip_s; a request that cannot fit an empty engine is an
error. (The GPU tests check the same loop with the real engines, bit for bit against single
solves.)
"""
import numpy as np
import pytest
import torch

import oracle
from paper_0812_2769_amd import problems, serve


class OracleEngine:
    def __init__(self, max_rows, max_systems, check_every=8, graph=False, device=None,
                 method="bicgstab", m=20, precision="fp64"):
        self.max_rows, self.max_systems, self.k = max_rows, max_systems, check_every
        self.method, self.m = method, m
        self.active = {}     # tag -> [rows, chunks left, info]
        self.log = []

    def request_bytes(self, A, p=2):
        return 8 * (A.nnz + A.n)

    def submit_gs(self, A, b, x, p=2, tol=1e-8, *, tag, maxit=None, breakdown_eps=None):
        rows = -(-A.n // 256) * 256
        used = sum(v[0] for v in self.active.values())
        if len(self.active) >= self.max_systems or used + rows > self.max_rows:
            return False
        xo, io = solve_alone(A, b.numpy(), self.method, self.m, tol)
        x.copy_(torch.from_numpy(xo))
        per_chunk = self.m if self.method == "gmres" else self.k
        self.active[tag] = [rows, max(1, -(-io.iters // per_chunk)), io]
        self.log.append(("admit", tag))
        return True

    def run(self, chunks=1):
        for v in self.active.values():
            v[1] -= chunks

    def poll(self, wait=True):
        done = [(t, v[2]) for t, v in self.active.items() if v[1] <= 0]
        for t, _ in done:
            del self.active[t]
            self.log.append(("done", t))
        return done

    def close(self):
        pass


def solve_alone(P, b, method, m, tol):
    vo, bo, _, _ = oracle.gs_scale(P, b, 2)
    S = P.copy()
    S.val, S.b = vo, bo
    if method == "gmres":
        return oracle.gmres(S, bo, m=m, tol=tol)
    return oracle.bicgstab(S, bo, tol=tol)


def make_requests(count, seed=3, spacing=0.0):
    specs = problems.batch_specs(count, seed=seed, n_min=6, n_max=14)
    reqs = []
    for i, sp in enumerate(specs):
        P = problems.batch_system(sp)
        reqs.append(serve.Request(tag=i, arrival=i * spacing, A=P, b=torch.from_numpy(P.b),
                                  method="gmres" if i % 4 == 3 else "bicgstab", m=10,
                                  tol=1e-8))
    return reqs


def test_every_request_served_once_with_its_alone_result():
    reqs = make_requests(12)
    rows = max(-(-r.A.n // 256) * 256 for r in reqs)
    srv = serve.Server(2 * rows, 2, graph=False, m_max=10, device="cpu", gmres_mode="engine",
                       gmres_engine_rows=rows, gmres_engine_systems=1,
                       engine_factory=OracleEngine)
    done = srv.serve(reqs, realtime=False)
    srv.close()
    assert sorted(d.tag for d in done) == list(range(len(reqs)))
    for d in done:
        r = reqs[d.tag]
        assert d.method == r.method
        xo, io = solve_alone(r.A, r.b.numpy(), r.method, r.m, r.tol)
        assert np.array_equal(d.x.numpy(), xo)
        assert d.info.iters == io.iters and d.info.status == io.status
        assert d.arrival <= d.admitted <= d.finished
    log = srv.engine.log
    first_done = next(i for i, (e, _) in enumerate(log) if e == "done")
    assert any(e == "admit" for e, _ in log[first_done:])   # retirements free room mid-run


def test_admission_waits_for_arrival():
    reqs = make_requests(6, seed=4, spacing=0.02)
    rows = max(-(-r.A.n // 256) * 256 for r in reqs)
    srv = serve.Server(4 * rows, 4, graph=False, m_max=10, device="cpu", gmres_mode="engine",
                       gmres_engine_rows=2 * rows, gmres_engine_systems=2,
                       engine_factory=OracleEngine)
    done = srv.serve(reqs, realtime=True)
    srv.close()
    assert len(done) == len(reqs)
    for d in done:
        assert d.admitted >= d.arrival - 1e-6


def test_request_larger_than_engine_is_an_error():
    reqs = [r for r in make_requests(4) if r.method == "bicgstab"]
    srv = serve.Server(128, 2, graph=False, m_max=10, device="cpu",
                       engine_factory=OracleEngine)
    with pytest.raises(ValueError):
        srv.serve(reqs, realtime=False)
    srv.close()


class Memory:
    """Stand-in free-memory probe: a fixed capacity minus what admitted, unfinished requests
    hold (their engine buffers and x), as the server charges them."""

    def __init__(self, capacity):
        self.capacity = capacity
        self.engines = []

    def __call__(self):
        used = sum(8 * (v[3].nnz + v[3].n) + 8 * v[3].n
                   for e in self.engines for v in e.active.values())
        return self.capacity - used


class MemEngine(OracleEngine):
    """The oracle stand-in, also keeping each active request's matrix for the memory probe."""

    def __init__(self, *a, memory=None, **k):
        super().__init__(*a, **k)
        memory.engines.append(self)

    def submit_gs(self, A, b, x, p=2, tol=1e-8, *, tag, maxit=None, breakdown_eps=None):
        ok = super().submit_gs(A, b, x, p, tol, tag=tag)
        if ok:
            self.active[tag].append(A)
        return ok


def bicg_requests(count, seed, spacing=0.0):
    return [r for r in make_requests(count, seed=seed, spacing=spacing)
            if r.method == "bicgstab"]


def test_free_memory_defers_admission_until_retirements():
    reqs = bicg_requests(16, seed=5)
    sizes = [8 * (r.A.nnz + r.A.n) + 8 * r.A.n for r in reqs]
    reserve = 100
    capacity = max(max(sizes), sum(sizes) // 3) + reserve   # a third of the set at a time
    mem = Memory(capacity)
    rows = sum(-(-r.A.n // 256) * 256 for r in reqs)       # rows and slots for all of them
    srv = serve.Server(rows, 32, graph=False, m_max=10, device="cpu",
                       engine_factory=lambda *a, **k: MemEngine(*a, memory=mem, **k),
                       free_bytes=mem, reserve_bytes=reserve)
    peak_used = 0
    orig_run = srv.engine.run

    def run(chunks=1):
        nonlocal peak_used
        peak_used = max(peak_used, capacity - mem())
        return orig_run(chunks)

    srv.engine.run = run
    done = srv.serve(reqs, realtime=False)
    srv.close()
    assert sorted(d.tag for d in done) == sorted(r.tag for r in reqs)
    assert peak_used <= capacity - reserve     # never more admitted than the memory holds
    assert srv.gate.deferred > 0               # and requests did wait for memory
    for d in done:                      # deferral changes no result
        r = next(q for q in reqs if q.tag == d.tag)
        xo, io = solve_alone(r.A, r.b.numpy(), r.method, r.m, r.tol)
        assert np.array_equal(d.x.numpy(), xo)


def _overtaking_setup(max_skip_s):
    # a small request, then a large one that does not fit beside it, then small ones
    small = [r for r in bicg_requests(16, seed=8) if r.A.n <= 256][:4]
    big = max(bicg_requests(16, seed=9), key=lambda r: r.A.n)
    assert big.A.n > 256 and len(small) == 4
    order = [small[0], big] + small[1:]
    reqs = [serve.Request(tag=i, arrival=0.0, A=r.A, b=r.b, method="bicgstab", tol=1e-8)
            for i, r in enumerate(order)]
    rows = -(-big.A.n // 256) * 256
    srv = serve.Server(rows, 8, graph=False, m_max=10, device="cpu",
                       engine_factory=OracleEngine, max_skip_s=max_skip_s)
    done = srv.serve(reqs, realtime=False)
    srv.close()
    assert sorted(d.tag for d in done) == list(range(len(reqs)))
    return [t for e, t in srv.engine.log if e == "admit"]


def test_smaller_requests_overtake_one_that_does_not_fit():
    admits = _overtaking_setup(max_skip_s=60.0)
    assert admits.index(2) < admits.index(1)   # a later small request went ahead of the big one


def test_no_overtaking_once_the_oldest_has_waited_max_skip():
    admits = _overtaking_setup(max_skip_s=-1.0)
    assert admits == sorted(admits)            # strict arrival order
