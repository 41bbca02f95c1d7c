"""Measured choice of the batch engine's launch shape and chunk length (the autotuner).

Two choices change how fast an FP64 Bi-CGSTAB engine runs but never its results (every choice
gives the same bits):
- the row-block shape of its streaming launches: one or two 256-row tiles per workgroup (two
  tiles keep both tiles' stencil loads in flight in one workgroup, halve the workgroup count,
  and need more registers per thread);
- the chunk length `check_every`, the iterations between host status reads: short chunks
  retire finished systems and admit waiting ones sooner but pay a host round trip (status
  copy, poll, upload) per chunk; long chunks let finished systems idle until the chunk ends.
Which is best depends on the batch and the device, so it is measured: every candidate runs the
same batch for its first iterations (all systems resident, the regime that dominates the batch
time; a small sample would leave the device underfilled and favour other shapes), and the
fastest wins.
Mixed-precision engines use two tiles (FP32 loads carry half the bytes) and FP64 GMRES engines
one (the single solver's partial sums), so only the chunk length is theirs to tune, and GMRES
engines run one restart cycle per chunk.
"""
import itertools
import time
from typing import Dict, List, Sequence

import torch

from . import gsk


def time_batch(systems: Sequence[dict], check_every: int, tol: float = 1e-8,
               device="cuda", tile_units: int = 1, maxit=None) -> float:
    """Seconds to run `systems` (dicts with an unscaled stencil or CSR matrix "S", a right-hand
    side "b" and row count "n") through GS(2) + Bi-CGSTAB (at most maxit iterations each) in
    one engine of that shape and chunk length."""
    unit = 256 * tile_units
    rows = sum((s["n"] + unit - 1) // unit * unit for s in systems)
    eng = gsk.Engine(rows, len(systems), check_every=check_every, graph=True, device=device,
                     tile_units=tile_units)
    xs = [torch.zeros_like(s["b"]) for s in systems]
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()   # graph captures count: the engine pays them too
        for i, s in enumerate(systems):
            assert eng.submit_gs(s["S"], s["b"], xs[i], p=2, tol=tol, tag=i, maxit=maxit)
        left = len(systems)
        while left:
            eng.run(1)
            left -= len(eng.poll(wait=True))
        torch.cuda.synchronize()
        return time.perf_counter() - t0
    finally:
        eng.close()


def tune_engine(systems: Sequence[dict], shapes: Sequence[int] = (1, 2),
                chunks: Sequence[int] = (4, 8, 16, 32), sample=None, tol: float = 1e-8,
                device="cuda", maxit: int = 48) -> Dict:
    """Times the batch (or its first `sample` systems) for at most `maxit` iterations per
    system with every (tiles per workgroup, chunk length) candidate and returns
    {"best": (units, chunk), "seconds": {(units, chunk): s}, "sample": count,
    "maxit": maxit}. Chunk lengths must be even (graph replay)."""
    part: List[dict] = list(systems if sample is None else systems[:sample])
    secs = {}
    for units, k in itertools.product(shapes, chunks):
        if k < 2 or k % 2:
            raise ValueError("chunk lengths must be even and >= 2")
        if units not in (1, 2):
            raise ValueError("tiles per workgroup must be 1 or 2")
        secs[(int(units), int(k))] = time_batch(part, int(k), tol, device, int(units), maxit)
    best = min(secs, key=secs.get)
    return {"best": best, "seconds": secs, "sample": len(part), "maxit": maxit}


def tune_check_every(systems: Sequence[dict], candidates: Sequence[int] = (4, 8, 16, 32),
                     sample=None, tol: float = 1e-8, device="cuda", maxit: int = 48) -> Dict:
    """The chunk length alone (one tile per workgroup): {"best": k, "seconds": {k: s}}."""
    t = tune_engine(systems, (1,), candidates, sample, tol, device, maxit)
    return {"best": t["best"][1], "seconds": {k: v for (_, k), v in t["seconds"].items()},
            "sample": t["sample"]}
