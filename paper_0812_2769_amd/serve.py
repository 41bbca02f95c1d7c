"""A solve server with continuous batching on one GPU.

Requests arrive over time (each an unscaled system, a method and a tolerance). The server:
- admits Bi-CGSTAB requests into the batched engine (gsk_engine_*) as soon as the engine has
  room (rows and a slot) and the device has the request's memory free, GS(2) included, so
  requests that arrive while others are on the GPU join the running batch at the next chunk;
- runs GMRES(m) requests either on a few lanes (each a host thread with a stream and
  workspaces of its own, one solve at a time) that take requests from one queue, or in a
  GMRES engine of their own (FP64 or mixed precision) on its own stream and host thread, so
  GMRES solves overlap each other and the Bi-CGSTAB engine's launches on the device;
- keeps every request's Krylov state on the device until it is done, and records arrival,
  admission and completion times.

Admission by free HBM. Engines hold their vectors in one workspace each; the server sizes
them from the device's free memory when no size is given (a fraction of it, split between the
Bi-CGSTAB and GMRES engines). Each request also needs memory of its own (the GS(2) outputs,
x, an FP32 matrix copy in a mixed engine), allocated when it is admitted: a request is
admitted only while the device's free memory (what the HIP runtime reports, plus what torch's
allocator holds unused) stays above a reserve after it. A request that does not fit waits;
requests behind it that fit are admitted meanwhile, unless the oldest waiting request has
waited longer than max_skip_s (then nothing overtakes it, so a large request cannot starve).

Each Bi-CGSTAB result is bit-for-bit the result of the same solve alone (the engine's
guarantee); each GMRES result is the single-solve path itself (lanes) or equal to it (engine).
"""
import collections
import dataclasses
import queue
import threading
import time
from typing import Callable, List, Optional

import torch

from . import gsk


@dataclasses.dataclass
class Request:
    tag: int
    arrival: float                 # seconds after the start of the run
    A: object                      # CsrMatrix or StencilMatrix (unscaled)
    b: torch.Tensor
    method: str = "bicgstab"       # "bicgstab" or "gmres"
    m: int = 20
    tol: float = 1e-8
    csr: Optional[object] = None   # the CSR form, needed by the GMRES lane's GS(2)
    grid: Optional[tuple] = None   # (nx, ny, nz) for packing the GMRES lane's scaled matrix


@dataclasses.dataclass
class Done:
    tag: int
    method: str
    arrival: float
    admitted: float
    finished: float
    info: gsk.Info
    x: torch.Tensor

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def device_free_bytes(device) -> int:
    """Free device memory usable by new allocations: what the HIP runtime reports free
    (hipMemGetInfo) plus what torch's caching allocator holds but does not use."""
    free, _ = torch.cuda.mem_get_info(device)
    cached = torch.cuda.memory_reserved(device) - torch.cuda.memory_allocated(device)
    return int(free) + max(0, int(cached))


class MemoryGate:
    """Admission by free device memory: fits(nbytes) while free - nbytes >= reserve.
    free_bytes() is the probe (device_free_bytes on a GPU; the host tests pass a stand-in)."""

    def __init__(self, free_bytes: Callable[[], int], reserve: int):
        self.free_bytes = free_bytes
        self.reserve = int(reserve)
        self.deferred = 0      # admissions refused for memory

    def fits(self, nbytes: int) -> bool:
        ok = self.free_bytes() - int(nbytes) >= self.reserve
        if not ok:
            self.deferred += 1
        return ok


def request_bytes(engine, req: Request) -> int:
    """Device bytes a request allocates when admitted: its engine's per-request buffers
    (Engine.request_bytes; an engine without it is charged 8 bytes per matrix value and row)
    plus x."""
    A = req.A
    fn = getattr(engine, "request_bytes", None)
    if fn is not None:
        nbytes = fn(A)
    else:
        vals = A.nnz if hasattr(A, "nnz") else A.n
        nbytes = 8 * (vals + A.n)
    return int(nbytes) + 8 * A.n


class GmresLane(threading.Thread):
    """Solves GMRES requests from a shared queue one at a time on its own stream: GS(2),
    packing, GMRES(m)."""

    def __init__(self, q: queue.Queue, device, t0: float, max_rows: int, m_max: int,
                 on_done: Callable):
        super().__init__(daemon=True)
        self.q = q
        self.error = None
        self.stream = torch.cuda.Stream(device)
        self.t0 = t0
        self.on_done = on_done
        self.device = device
        self.abort = threading.Event()
        with torch.cuda.stream(self.stream):
            self.ws_gs = gsk.workspace(gsk.METHOD_GS, max_rows, 0, device)
            self.ws = gsk.workspace(gsk.METHOD_GMRES, max_rows, m_max, device)

    def run(self):
        while True:
            item = self.q.get()
            if item is None or self.abort.is_set():
                self.q.task_done()
                if item is None:
                    return
                continue
            try:
                req, admitted = item
                with torch.cuda.stream(self.stream):
                    A = req.csr
                    As, bs, _, _ = gsk.gs_scale(A, req.b, 2, want_norms=False, ws=self.ws_gs)
                    M = gsk.stencil_from_csr(As, *req.grid, ws=self.ws_gs) if req.grid else As
                    ws = self.ws[: gsk.workspace_bytes(gsk.METHOD_GMRES, A.n, req.m)]
                    x, info = gsk.gmres(M, bs, m=req.m, tol=req.tol, ws=ws)
                self.stream.synchronize()
                self.on_done(Done(req.tag, "gmres", req.arrival, admitted,
                                  time.perf_counter() - self.t0, info, x))
            except BaseException as e:   # reported by the server loop
                self.error = e
            finally:
                self.q.task_done()

    def close(self):
        pass


class GmresEngineWorker(threading.Thread):
    """Serves GMRES(m) requests through a GMRES engine of its own (its own stream): admits them
    as rows, slots and device memory free up (GS(2) inside the engine), runs one cycle per
    chunk, and reports each finished request. Results equal gsk_gmres (or gsk_gmres_mixed) on
    the same system. Setting `abort` makes it stop between chunks without draining its
    requests."""

    def __init__(self, q: queue.Queue, device, t0: float, max_rows: int, max_systems: int,
                 m: int, precision: str, graph: bool, on_done: Callable,
                 engine_factory: Callable = gsk.Engine, gate: Optional[MemoryGate] = None):
        super().__init__(daemon=True)
        self.q = q
        self.error = None
        self.t0 = t0
        self.on_done = on_done
        self.m = m
        self.gate = gate
        self.abort = threading.Event()
        self.engine = engine_factory(max_rows, max_systems, graph=graph, device=device,
                                     method="gmres", m=m, precision=precision)

    def run(self):
        waiting = collections.deque()
        inflight = {}
        closing = False
        try:
            while not (closing and not waiting and not inflight):
                if self.abort.is_set():
                    return
                # take new requests; block only when there is nothing else to do
                block = not waiting and not inflight and not closing
                while True:
                    try:
                        item = self.q.get(block=block, timeout=0.05 if block else None)
                    except queue.Empty:
                        break
                    block = False
                    if item is None:
                        closing = True
                        continue
                    waiting.append(item)
                while waiting:
                    req, admitted = waiting[0]
                    if req.m != self.m:
                        raise ValueError(f"request m={req.m} on a GMRES({self.m}) engine")
                    if self.gate is not None and inflight and \
                            not self.gate.fits(request_bytes(self.engine, req)):
                        break
                    x = torch.zeros_like(req.b)
                    if not self.engine.submit_gs(req.A, req.b, x, p=2, tol=req.tol,
                                                 tag=req.tag):
                        if not inflight:   # an empty engine that cannot take it never will
                            raise ValueError(f"request {req.tag} ({req.A.n} rows) does not "
                                             "fit the GMRES engine")
                        break
                    inflight[req.tag] = (req, admitted, x)
                    waiting.popleft()
                if inflight:
                    self.engine.run(1)
                    for tag, info in self.engine.poll(wait=True):
                        req, adm, x = inflight.pop(tag)
                        self.on_done(Done(tag, "gmres", req.arrival, adm,
                                          time.perf_counter() - self.t0, info, x))
        except BaseException as e:   # reported by the server loop
            self.error = e

    def close(self):
        self.engine.close()


class Server:
    def __init__(self, max_rows: int = 0, max_systems: int = 256, check_every: int = 8,
                 graph: bool = True, gmres_rows: int = 0, m_max: int = 20, device="cuda",
                 gmres_lanes: int = 4, gmres_mode: str = "lanes",
                 gmres_precision: str = "fp64", gmres_engine_rows: int = 0,
                 gmres_engine_systems: int = 64, engine_factory: Callable = gsk.Engine,
                 tile_units: int = 0, free_bytes: Optional[Callable[[], int]] = None,
                 hbm_fraction: float = 0.25, reserve_bytes: int = 2 << 30,
                 max_rows_cap: int = 1 << 28, max_skip_s: float = 1.0):
        """max_rows / gmres_engine_rows: the engines' row capacity; 0 sizes them from free
        device memory (hbm_fraction of it, half to each engine when GMRES runs in an engine,
        at most max_rows_cap rows each). gmres_mode "lanes": GMRES requests run one at a time
        on gmres_lanes host threads (workspaces for gmres_rows rows, any m <= m_max).
        "engine": they run in a GMRES(m_max) engine (gmres_precision "fp64" or "mixed").
        tile_units: the Bi-CGSTAB engine's tiles per workgroup. free_bytes(): the free-memory
        probe (device_free_bytes by default); requests are admitted while free memory after
        them stays above reserve_bytes. A request that does not fit is overtaken by later
        ones that fit until it has waited max_skip_s. engine_factory(max_rows, max_systems,
        **options) builds the engines (gsk.Engine; the scheduler's host-side tests pass a
        stand-in with the same submit_gs / run / poll / close methods)."""
        self.device = torch.device(device)
        self.engine_factory = engine_factory
        if free_bytes is not None:
            probe = free_bytes
        elif self.device.type == "cuda":
            probe = lambda: device_free_bytes(self.device)   # noqa: E731
        else:
            probe = lambda: 1 << 62   # noqa: E731  (host stand-in engines: memory is no limit)
        self.gate = MemoryGate(probe, reserve_bytes)
        if gmres_mode not in ("lanes", "engine"):
            raise ValueError("gmres_mode must be 'lanes' or 'engine'")
        self.sizing = None
        if not max_rows or (gmres_mode == "engine" and not gmres_engine_rows):
            budget = max(0, probe() - reserve_bytes) * hbm_fraction
            parts = 2 if gmres_mode == "engine" else 1
            bpr_b = self._bytes_per_row("bicgstab", "fp64", 0)
            bpr_g = self._bytes_per_row("gmres", gmres_precision, m_max)
            if not max_rows:
                max_rows = max(256, min(max_rows_cap, int(budget / parts / bpr_b)))
            if gmres_mode == "engine" and not gmres_engine_rows:
                gmres_engine_rows = max(256, min(max_rows_cap, int(budget / parts / bpr_g)))
            self.sizing = {"free_bytes": probe(), "budget_bytes": int(budget),
                           "bicgstab_rows": int(max_rows),
                           "gmres_rows": int(gmres_engine_rows) if gmres_mode == "engine"
                           else None}
        opts = {"tile_units": tile_units} if tile_units else {}
        self.engine = engine_factory(max_rows, max_systems, check_every=check_every, graph=graph,
                                     device=self.device, **opts)
        self.max_rows = max_rows
        self.gmres_rows = gmres_rows
        self.m_max = m_max
        self.gmres_lanes = max(1, int(gmres_lanes))
        self.gmres_mode = gmres_mode
        self.gmres_precision = gmres_precision
        self.gmres_engine_rows = gmres_engine_rows or max(gmres_rows, 1)
        self.gmres_engine_systems = gmres_engine_systems
        self.graph = graph
        self.max_skip_s = max_skip_s

    def _bytes_per_row(self, method, precision, m):
        fn = getattr(self.engine_factory, "workspace_bytes_per_row", None)
        return fn(method, precision, m) if fn is not None else 64.0

    def serve(self, requests: List[Request], realtime: bool = True) -> List[Done]:
        """Serve the requests (sorted by arrival). With realtime, a request is visible only
        once the wall clock has passed its arrival time."""
        reqs = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting: List[Request] = []
        done: List[Done] = []
        lock = threading.Lock()
        t0 = time.perf_counter()
        lanes = []
        gq = queue.Queue()
        if any(r.method == "gmres" for r in reqs):
            def finished(d):
                with lock:
                    done.append(d)
            if self.gmres_mode == "engine":
                lanes = [GmresEngineWorker(gq, self.device, t0, self.gmres_engine_rows,
                                           self.gmres_engine_systems, self.m_max,
                                           self.gmres_precision, self.graph, finished,
                                           self.engine_factory, self.gate)]
            else:
                lanes = [GmresLane(gq, self.device, t0, max(self.gmres_rows, 1), self.m_max,
                                   finished) for _ in range(self.gmres_lanes)]
            for lane in lanes:
                lane.start()
        inflight = {}     # engine tag -> (request, admitted time, x)
        n_total = len(reqs)
        failed = False
        try:
            while True:
                now = time.perf_counter() - t0
                while reqs and (not realtime or reqs[0].arrival <= now):
                    r = reqs.popleft()
                    if r.method == "gmres":
                        gq.put((r, now))
                    else:
                        waiting.append(r)
                self._admit(waiting, inflight, now)
                if inflight:
                    self.engine.run(1)
                    for tag, info in self.engine.poll(wait=True):
                        r, adm, x = inflight.pop(tag)
                        with lock:
                            done.append(Done(tag, "bicgstab", r.arrival, adm,
                                             time.perf_counter() - t0, info, x))
                else:
                    if not reqs and not waiting:
                        with lock:
                            if len(done) >= n_total:
                                break
                        time.sleep(1e-3)   # the GMRES workers are still solving
                    if reqs and realtime:
                        time.sleep(max(0.0, min(1e-3, reqs[0].arrival - now)))
                for lane in lanes:
                    if lane.error is not None:
                        raise RuntimeError("GMRES lane failed") from lane.error
                with lock:
                    if len(done) >= n_total:
                        break
        except BaseException:
            failed = True
            raise
        finally:
            for lane in lanes:
                if failed:
                    lane.abort.set()
                gq.put(None)
            for lane in lanes:
                lane.join(timeout=60)
                if lane.is_alive():
                    # still inside a device call: leave its engine alone (closing it under
                    # a running worker would free memory the worker still uses)
                    continue
                lane.close()
        return done

    def _admit(self, waiting: List[Request], inflight: dict, now: float) -> None:
        """Admit waiting Bi-CGSTAB requests that fit the engine and the free memory, in
        arrival order; a request that does not fit is overtaken by later ones until it has
        waited max_skip_s."""
        k = 0
        while k < len(waiting):
            r = waiting[k]
            fits = not inflight or self.gate.fits(request_bytes(self.engine, r))
            x = None
            if fits:
                x = torch.zeros_like(r.b)
                fits = self.engine.submit_gs(r.A, r.b, x, p=2, tol=r.tol, tag=r.tag)
                if not fits and not inflight:   # an empty engine that cannot take it never will
                    raise ValueError(f"request {r.tag} ({r.A.n} rows) does not fit the engine")
            if fits:
                inflight[r.tag] = (r, now, x)
                waiting.pop(k)
                continue
            if k == 0 and now - r.arrival > self.max_skip_s:
                return      # the oldest request has waited long enough: nothing overtakes it
            k += 1

    def close(self):
        self.engine.close()
