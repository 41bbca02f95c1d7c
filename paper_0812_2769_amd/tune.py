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
An FP64 Bi-CGSTAB engine can also take a shape per size class (2D stencils and CSR, 3D stencils
under 2^18 rows, larger 3D stencils), each class with launches of its own: tune_classes times
each class alone with every shape, then the chunk length on the whole batch.
Mixed-precision engines use two tiles (FP32 loads carry half the bytes) and FP64 GMRES engines
one (the single solver's partial sums), so only the chunk length is theirs to tune
(tune_mixed_chunk), and GMRES engines run one restart cycle per chunk.
"""
import itertools
import time
from typing import Dict, List, Sequence

import torch

from . import gsk


def time_batch(systems: Sequence[dict], check_every: int, tol: float = 1e-8,
               device="cuda", tile_units: int = 1, maxit=None, class_shapes=None,
               precision: str = "fp64") -> float:
    """Seconds to run `systems` (dicts with an unscaled stencil or CSR matrix "S", a right-hand
    side "b" and row count "n") through GS(2) + Bi-CGSTAB (at most maxit iterations each) in
    one engine of that shape (tiles per workgroup, or a shape per size class) and chunk
    length."""
    unit = 512 if (tile_units == 2 or class_shapes or precision == "mixed") else 256
    rows = sum((s["n"] + unit - 1) // unit * unit for s in systems)
    eng = gsk.Engine(rows, len(systems), check_every=check_every, graph=True, device=device,
                     tile_units=tile_units if precision == "fp64" else 0,
                     class_shapes=class_shapes, precision=precision)
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


def tune_classes(systems: Sequence[dict], shapes: Sequence[str] = ("tile", "pair_tile_u", "pair"),
                 chunks: Sequence[int] = (8, 16, 32), tol: float = 1e-8, device="cuda",
                 maxit: int = 48, repeats: int = 2) -> Dict:
    """Per-size-class launch shapes of an FP64 Bi-CGSTAB engine, then its chunk length.

    In an engine with size classes every class has launches of its own, which run on the
    device one after another; so each class's systems are timed alone (all resident, first
    `maxit` iterations) with every shape, best of `repeats`, and the fastest shape is the
    class's. The chunk length is then timed on the whole batch with those shapes. Returns
    {"class_shapes": {class: shape}, "chunk": k, "class_seconds": {class: {shape: s}},
    "class_systems": {class: count}, "class_rows": {class: rows}, "chunk_seconds": {k: s},
    "maxit": maxit}."""
    by_class: Dict[str, List[dict]] = {}
    for s in systems:
        by_class.setdefault(gsk.size_class(s["S"]), []).append(s)
    chosen, class_secs = {}, {}
    for c, part in sorted(by_class.items()):
        secs = {}
        for shape in shapes:
            secs[shape] = min(time_batch(part, 16, tol, device, maxit=maxit,
                                         class_shapes={c: shape}) for _ in range(repeats))
        class_secs[c] = secs
        chosen[c] = min(secs, key=secs.get)
    chunk_secs = {}
    for k in chunks:
        if k < 2 or k % 2:
            raise ValueError("chunk lengths must be even and >= 2")
        chunk_secs[int(k)] = min(time_batch(systems, int(k), tol, device, maxit=maxit,
                                            class_shapes=chosen) for _ in range(repeats))
    return {"class_shapes": chosen, "chunk": min(chunk_secs, key=chunk_secs.get),
            "class_seconds": class_secs,
            "class_systems": {c: len(v) for c, v in by_class.items()},
            "class_rows": {c: int(sum(s["n"] for s in v)) for c, v in by_class.items()},
            "chunk_seconds": chunk_secs, "maxit": maxit}


def tune_mixed_chunk(systems: Sequence[dict], chunks: Sequence[int] = (8, 16, 32),
                     tol: float = 1e-8, device="cuda", maxit: int = 48) -> Dict:
    """Chunk length of a mixed-precision Bi-CGSTAB engine (its launch shape is fixed: two
    tiles per workgroup, since FP32 loads carry half the bytes): {"chunk": k,
    "chunk_seconds": {k: s}}."""
    secs = {int(k): time_batch(systems, int(k), tol, device, maxit=maxit, precision="mixed")
            for k in chunks}
    return {"chunk": min(secs, key=secs.get), "chunk_seconds": secs, "maxit": maxit}
