"""A solve server with continuous batching on one GPU.

Requests arrive over time (each an unscaled system, a method and a tolerance). The server:
- admits Bi-CGSTAB requests into the batched engine (gsk_engine_*) as soon as its workspace
  has room (rows and a slot), GS(2) included, so requests that arrive while others are on the
  GPU join the running batch at the next chunk;
- runs GMRES(m) requests either on a few lanes (each a host thread with a stream and
  workspaces of its own, one solve at a time) that take requests from one queue, or in a
  GMRES engine of their own (FP64 or mixed precision) on its own stream and host thread, so
  GMRES solves overlap each other and the Bi-CGSTAB engine's launches on the device;
- keeps every request's Krylov state on the device until it is done, and records arrival,
  admission and completion times.

Each Bi-CGSTAB result is bit-for-bit the result of the same solve alone (the engine's
guarantee); each GMRES result is the single-solve path itself.
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
        with torch.cuda.stream(self.stream):
            self.ws_gs = gsk.workspace(gsk.METHOD_GS, max_rows, 0, device)
            self.ws = gsk.workspace(gsk.METHOD_GMRES, max_rows, m_max, device)

    def run(self):
        while True:
            item = self.q.get()
            if item is None:
                return
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


class GmresEngineWorker(threading.Thread):
    """Serves GMRES(m) requests through a GMRES engine of its own (its own stream): admits them
    as rows and slots free up (GS(2) inside the engine), runs one cycle per chunk, and reports
    each finished request. Results equal gsk_gmres (or gsk_gmres_mixed) on the same system."""

    def __init__(self, q: queue.Queue, device, t0: float, max_rows: int, max_systems: int,
                 m: int, precision: str, graph: bool, on_done: Callable,
                 engine_factory: Callable = gsk.Engine):
        super().__init__(daemon=True)
        self.q = q
        self.error = None
        self.t0 = t0
        self.on_done = on_done
        self.m = m
        self.engine = engine_factory(max_rows, max_systems, graph=graph, device=device,
                                     method="gmres", m=m, precision=precision)

    def run(self):
        waiting = collections.deque()
        inflight = {}
        closing = False
        try:
            while not (closing and not waiting and not inflight):
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
    def __init__(self, max_rows: int, max_systems: int, check_every: int = 8,
                 graph: bool = True, gmres_rows: int = 0, m_max: int = 20, device="cuda",
                 gmres_lanes: int = 4, gmres_mode: str = "lanes",
                 gmres_precision: str = "fp64", gmres_engine_rows: int = 0,
                 gmres_engine_systems: int = 64, engine_factory: Callable = gsk.Engine,
                 tile_units: int = 0):
        """gmres_mode "lanes": GMRES requests run one at a time on gmres_lanes host threads
        (workspaces for gmres_rows rows, any m <= m_max). "engine": they run in a GMRES(m_max)
        engine (gmres_precision "fp64" or "mixed") with room for gmres_engine_rows rows and
        gmres_engine_systems systems. tile_units: the Bi-CGSTAB engine's tiles per workgroup
        (0 or 1: one, 2: two; max_rows must then hold each system rounded up to 512 rows).
        engine_factory(max_rows, max_systems, **options) builds the engines (gsk.Engine; the
        scheduler's host-side tests pass a stand-in with the same submit_gs / run / poll /
        close methods)."""
        self.device = torch.device(device)
        self.engine_factory = engine_factory
        opts = {"tile_units": tile_units} if tile_units else {}
        self.engine = engine_factory(max_rows, max_systems, check_every=check_every, graph=graph,
                                     device=self.device, **opts)
        self.gmres_rows = gmres_rows
        self.m_max = m_max
        self.gmres_lanes = max(1, int(gmres_lanes))
        if gmres_mode not in ("lanes", "engine"):
            raise ValueError("gmres_mode must be 'lanes' or 'engine'")
        self.gmres_mode = gmres_mode
        self.gmres_precision = gmres_precision
        self.gmres_engine_rows = gmres_engine_rows or max(gmres_rows, 1)
        self.gmres_engine_systems = gmres_engine_systems
        self.graph = graph

    def serve(self, requests: List[Request], realtime: bool = True) -> List[Done]:
        """Serve the requests (sorted by arrival). With realtime, a request is visible only
        once the wall clock has passed its arrival time."""
        reqs = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting = collections.deque()
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
                                           self.engine_factory)]
            else:
                lanes = [GmresLane(gq, self.device, t0, max(self.gmres_rows, 1), self.m_max,
                                   finished) for _ in range(self.gmres_lanes)]
            for lane in lanes:
                lane.start()
        inflight = {}     # engine tag -> (request, admitted time, x)
        n_total = len(reqs)
        try:
            while True:
                now = time.perf_counter() - t0
                while reqs and (not realtime or reqs[0].arrival <= now):
                    waiting.append(reqs.popleft())
                # admit in arrival order; a request that does not fit waits for retirements
                while waiting:
                    r = waiting[0]
                    if r.method == "gmres":
                        gq.put((r, now))
                        waiting.popleft()
                        continue
                    x = torch.zeros_like(r.b)
                    if not self.engine.submit_gs(r.A, r.b, x, p=2, tol=r.tol, tag=r.tag):
                        if not inflight:   # an empty engine that cannot take it never will
                            raise ValueError(f"request {r.tag} ({r.A.n} rows) does not fit "
                                             "the engine")
                        break
                    inflight[r.tag] = (r, now, x)
                    waiting.popleft()
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
        finally:
            for _ in lanes:
                gq.put(None)
            for lane in lanes:
                lane.join(timeout=60)
                if isinstance(lane, GmresEngineWorker):
                    lane.close()
        return done

    def close(self):
        self.engine.close()
