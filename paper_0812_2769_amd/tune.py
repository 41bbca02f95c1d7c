"""Measured choice of the batch engine's chunk length.

A Bi-CGSTAB engine runs `check_every` iterations per chunk between host status reads. Short
chunks retire finished systems and admit waiting ones sooner but pay a host round trip (status
copy, poll, upload) per chunk; long chunks let finished systems idle until the chunk ends. The
best length depends on the batch (sizes, iteration spread), so it is measured: each candidate
solves the same sample of the batch once, and the fastest wins. GMRES engines run one restart
cycle per chunk and have nothing to tune here.

Tile shapes are not tuned: two 256-row tiles per workgroup were measured against one on the
FP64 kernels (equal or slower), and FP32 data need two (the single solver's finding), so the
engine fixes them by precision.
"""
import time
from typing import Dict, List, Sequence

import torch

from . import gsk


def time_batch(systems: Sequence[dict], check_every: int, tol: float = 1e-8,
               device="cuda") -> float:
    """Seconds to solve `systems` (dicts with an unscaled stencil or CSR matrix "S", a right-hand
    side "b" and row count "n") with GS(2) + Bi-CGSTAB in one engine of that chunk length."""
    rows = sum((s["n"] + 255) // 256 * 256 for s in systems)
    eng = gsk.Engine(rows, len(systems), check_every=check_every, graph=True, device=device)
    xs = [torch.zeros_like(s["b"]) for s in systems]
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()   # graph captures count: the engine pays them too
        for i, s in enumerate(systems):
            assert eng.submit_gs(s["S"], s["b"], xs[i], p=2, tol=tol, tag=i)
        left = len(systems)
        while left:
            eng.run(1)
            left -= len(eng.poll(wait=True))
        torch.cuda.synchronize()
        return time.perf_counter() - t0
    finally:
        eng.close()


def tune_check_every(systems: Sequence[dict], candidates: Sequence[int] = (4, 8, 16, 32),
                     sample: int = 64, tol: float = 1e-8, device="cuda") -> Dict:
    """Times a batch of the first `sample` systems with every candidate chunk length (even
    values, for graph replay) and returns {"best": k, "seconds": {k: s}}."""
    part: List[dict] = list(systems[:sample])
    secs = {}
    for k in candidates:
        if k < 2 or k % 2:
            raise ValueError("chunk lengths must be even and >= 2")
        secs[int(k)] = time_batch(part, int(k), tol, device)
    best = min(secs, key=secs.get)
    return {"best": best, "seconds": secs, "sample": len(part)}
