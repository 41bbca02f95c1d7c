"""A solve server with continuous batching on one GPU.

Requests arrive over time (each an unscaled system, a method and a tolerance). The server:
- admits Bi-CGSTAB requests into the batched engine (gsk_engine_*) as soon as its workspace
  has room (rows and a slot), GS(2) included, so requests that arrive while others are on the
  GPU join the running batch at the next chunk;
- runs GMRES(m) requests on a few lanes (each a host thread with a stream and workspaces of
  its own) that take requests from one queue, so GMRES solves overlap each other and the
  engine's launches on the device;
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


class Server:
    def __init__(self, max_rows: int, max_systems: int, check_every: int = 8,
                 graph: bool = True, gmres_rows: int = 0, m_max: int = 20, device="cuda",
                 gmres_lanes: int = 4):
        self.device = torch.device(device)
        self.engine = gsk.Engine(max_rows, max_systems, check_every=check_every, graph=graph,
                                 device=self.device)
        self.gmres_rows = gmres_rows
        self.m_max = m_max
        self.gmres_lanes = max(1, int(gmres_lanes))

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
                        if lanes:
                            gq.join()   # every lane calls task_done, also after an error
                        with lock:
                            if len(done) >= n_total:
                                break
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
        return done

    def close(self):
        self.engine.close()
