"""Benchmark: GS(2) + Krylov solves on one MI355X; one JSON line on stdout.

Default workload (`--workload batch512`): the batch of 512 independent convection-diffusion
systems (seeded, synthetic: for each system, from numpy default_rng(1004), d uniform in {2,3},
side N uniform in [32, 96] interior nodes, a = 10^U(2,6) on a random box and 1 elsewhere,
convection components U(0,30), b = A u* with u* the sine product; 265 2D and 247 3D systems,
81.8 M rows in all). The systems are uploaded unscaled (5/7-point coefficient planes) before
timing. One step = one batch: every system is submitted to the batch engine with a GS(2) stage
and solved by Bi-CGSTAB to a relative residual below 1e-8 (the stop test on the GS(2)-scaled
system, verified with the true residual); chunks of iterations are replayed from HIP graphs.
  value       converged solves per second over the timed steps (systems that end MAXIT,
              STAGNATED or BREAKDOWN are not counted; their statuses and residuals are listed)
  latency     p50/p99 over the systems of the timed steps, from the batch's submission to
              the system's retirement
  roofline    k_batch_p (the dominant launch: p update, A p, two dot products): algorithmic
              bytes of the timed launches / their HIP-event durations, every 4th chunk of the
              timed steps enqueued without its graph and its P launches timed
  cpu_baseline  the C oracle (GS(2) + Bi-CGSTAB) on a seeded sample of the systems, one
              system per host thread
  extras      the 80^3 slabs system's four solves (GS(1|2) x Bi-CGSTAB | GMRES(30), tol 1e-10;
              cache-resident: its bandwidth is fabric bandwidth) and the 160^3 checkerboard
              system (HBM-resident): the FP64 k_gmres_a roofline over two GMRES(30) cycles and
              the GS(2) + Bi-CGSTAB solve to 1e-8.

Other modes:
  --workload slabs80     the 80^3 system's four solves (GS(1|2) x Bi-CGSTAB | GMRES(30)).
  --workload checker160  the 160^3 checkerboard system: GS(2) + Bi-CGSTAB to 1e-8 (value =
                         its solves/s), and GMRES(30) in FP64 and in mixed precision run to the
                         10,000-step cap, with the relative residual they reach.
  --workload serving     Poisson arrivals through the solve server.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solves/s at 1e-8 rel. residual, Krylov HBM GB/s vs peak, p50/p99 latency"
HBM_PEAK_GBS = 8000.0
KERNEL_NAMES = {"gmres_a": "k_gmres_a (matrix product + CGS2 pass-1 dots)",
                "gmres_b": "k_gmres_b (CGS2 pass-1 update + pass-2 dots)",
                "gmres_c": "k_gmres_c (CGS2 pass-2 update + norm)",
                "bicg_p": "k_bicg_p (p update + matrix product + dots)",
                "bicg_s": "k_bicg_s (s + matrix product + dots)",
                "bicg_u": "k_bicg_u (x, r update + dots)",
                "residual": "k_*_residual (true residual)",
                "gmres_x": "k_gmres_x (x += V y)",
                "batch_p": "k_batch_p (batch engine: p update + matrix product + dots)",
                "batch_s": "k_batch_s (batch engine: s + matrix product + dots)",
                "batch_u": "k_batch_u (batch engine: x, r update + dots)"}

# Fabric (HBM + Infinity Cache) bytes per working launch of a kernel class, from two
# rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE; FETCH_SIZE scaled by 2.000 and WRITE_SIZE by
# 1.000 from a plain 512 MiB copy), recorded with the hash of the kernel sources they were
# measured on. A source change makes the figure stale and it is reported as null.
# Counter-measured HBM traffic (FETCH_SIZE x 2.000 + WRITE_SIZE, calibrated on a copy) of the
# dominant kernel per workload, as a ratio to the algorithmic bytes of the same launches
# (profiles/*_hbm_counters.md). A record applies while the kernel sources hash to the ones
# the counters were taken with.
GMRES_SOURCES = ["paper_0812_2769_amd/csrc/gmres.hip", "paper_0812_2769_amd/csrc/gmres_body.hpp",
                 "paper_0812_2769_amd/csrc/gsk_dev.hpp"]
BATCH_SOURCES = ["paper_0812_2769_amd/csrc/batch.hip", "paper_0812_2769_amd/csrc/bicg_batch.hpp",
                 "paper_0812_2769_amd/csrc/batch.hpp", "paper_0812_2769_amd/csrc/gsk_dev.hpp"]
TRAFFIC = [
    # the 512-system batch: P launches of full-batch iterations
    {"probe": "batch_p", "grid": None, "ratio": 8.536 / 8.491, "sources": BATCH_SOURCES,
     "sources_sha256_16": "31777f05ccd859a5"},
    # FP64 GMRES(30) on the 160^3 checkerboard: the A launches of two cycles
    {"probe": "gmres_a", "grid": 160, "ratio": 775.12 / 770.05, "sources": GMRES_SOURCES,
     "sources_sha256_16": "32fbb655b87db429"},
    # the 80^3 slabs (cache-resident): the A launches of the two GMRES(30) solves
    {"probe": "gmres_a", "grid": 80, "ratio": 96.14 / 96.03, "sources": GMRES_SOURCES,
     "sources_sha256_16": "32fbb655b87db429"},
]


def traffic_for(probe, grid, operator, bytes_per_launch):
    """Counter-measured HBM bytes per launch of the probed class (the record's ratio times the
    algorithmic bytes per launch), or None when no record matches the workload or the kernel
    sources have changed since the counters were taken."""
    import hashlib
    if operator != "stencil" or bytes_per_launch is None:
        return None
    for rec in TRAFFIC:
        if rec["probe"] != probe or rec["grid"] != grid or rec["ratio"] is None:
            continue
        h = hashlib.sha256()
        for f in rec["sources"]:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest()[:16] == rec["sources_sha256_16"]:
            return int(rec["ratio"] * bytes_per_launch)
    return None


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["batch512", "slabs80", "checker160", "serving"],
                    default="batch512")
    ap.add_argument("--gmres-lanes", type=int, default=4,
                    help="serving: host threads (each with its own stream) serving GMRES")
    ap.add_argument("--gmres-mode", choices=["lanes", "engine"], default="engine",
                    help="serving: GMRES requests on lanes or in a GMRES engine")
    ap.add_argument("--gmres-precision", choices=["fp64", "mixed"], default="mixed",
                    help="serving with --gmres-mode engine: the GMRES engine's precision "
                         "(mixed: FP32 Arnoldi cycles, FP64 restarts and stop test)")
    ap.add_argument("--tile-units", type=int, default=0,
                    help="batch512: tiles per workgroup (1 or 2) instead of measuring; serving: "
                         "the Bi-CGSTAB engine's tiles per workgroup")
    ap.add_argument("--chunk", type=int, default=0,
                    help="batch512: iterations per chunk instead of measuring")
    ap.add_argument("--no-tune", action="store_true",
                    help="batch512: one tile per workgroup and chunks of 8 instead of measuring")
    ap.add_argument("--class-shapes", default="",
                    help="batch512 (FP64 Bi-CGSTAB): launch shape per size class instead of "
                         "measuring, e.g. 2d=pair,3d_small=pair_tile_u,3d_large=pair_tile_u "
                         "(chunks of --chunk, default 16)")
    ap.add_argument("--batch-method", choices=["bicgstab", "gmres"], default="bicgstab",
                    help="batch512: the engine's solver (GMRES(20) with --precision)")
    ap.add_argument("--batch-count", type=int, default=512,
                    help="batch512: systems per batch (default 512)")
    ap.add_argument("--no-solo", action="store_true",
                    help="batch512: skip the one-at-a-time comparison")
    ap.add_argument("--no-extras", action="store_true",
                    help="batch512: skip the 80^3 and 160^3 figures")
    ap.add_argument("--cpu-sample-systems", type=int, default=96,
                    help="batch512: systems of the batch the CPU oracle solves for its baseline")
    ap.add_argument("--rates", default="50,100,200,500,1000,2000",
                    help="serving: Poisson arrival rates to sweep (requests/s)")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="serving: requests per rate")
    ap.add_argument("--gmres-share", type=float, default=0.5,
                    help="serving: fraction of GMRES(20) requests (the rest Bi-CGSTAB)")
    ap.add_argument("--serve-pool", type=int, default=128,
                    help="serving: systems drawn from the batch recipe that requests pick from")
    ap.add_argument("--grid", type=int, default=0,
                    help="N of the N^3 grid (default 80 for slabs80, 160 for checker160)")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64",
                    help="slabs80: GMRES solves in FP64 (default) or mixed precision; batch512: "
                         "the engine's precision")
    ap.add_argument("--checker-steps", type=int, default=0,
                    help="checker160: Arnoldi steps per GMRES solve (default: the 10,000 cap)")
    ap.add_argument("--operator", choices=["stencil", "csr"], default="stencil",
                    help="matrix form the solvers read: 7-point coefficient planes packed from "
                         "the scaled CSR matrix inside each solve (default), or the CSR matrix")
    ap.add_argument("--cpu-sample-iters", type=int, default=120,
                    help="slabs80/checker160: iterations per solver the CPU oracle runs for its "
                         "baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--probe", default="",
                    help="kernel class timed with HIP events during the timed steps ('none' to "
                         "time nothing; default batch_p for batch512, gmres_a otherwise)")
    ap.add_argument("--probe-every", type=int, default=4,
                    help="time every k-th launch (batch engine: every k-th chunk) of the probed "
                         "class (default 4)")
    ap.add_argument("--no-kernel-table", action="store_true",
                    help="slabs80: skip the extra untimed step per kernel class")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB MiB (reference for HBM "
                         "byte counters) and exit")
    return ap.parse_args(argv)


def pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo = int(k)
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def host_cpu():
    """The host's processor model and the cores this process may use."""
    model = None
    ids = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                key, _, val = line.partition(":")
                key = key.strip()
                if key == "model name" and model is None:
                    model = val.strip()
                elif key in ("cpu family", "model") and key not in ids:
                    ids[key] = val.strip()
                elif not line.strip() and model is not None:
                    break   # first processor's block read
    except OSError:
        pass
    if model is not None and ids:
        # the model name can be generic under virtualisation; family and model numbers
        # identify the core generation
        model = f"{model} (family {ids.get('cpu family', '?')}, model {ids.get('model', '?')})"
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return {"model": model, "cores_available": cores, "nproc": os.cpu_count()}


def cpu_threads():
    """Worker threads for the oracle baseline: the cores this process may use, at most 16 (the
    host share of one GPU)."""
    return max(1, min(16, host_cpu()["cores_available"]))


def achieved(pr):
    if pr is None or pr["total_ms"] <= 0 or pr["busy_launches"] == 0:
        return None
    return {"achieved_GBs": round(pr["bytes"] / (pr["total_ms"] * 1e-3) / 1e9, 1),
            "avg_launch_us": round(1e3 * pr["total_ms"] / pr["busy_launches"], 3),
            "bytes_per_launch": round(pr["bytes"] / pr["busy_launches"]),
            "timed_launches": pr["launches"], "busy_launches": pr["busy_launches"]}


def roofline_of(a, probe, every, traffic=None, note=None):
    return {"bound": "hbm", "achieved": a["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(a["achieved_GBs"] / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": KERNEL_NAMES.get(probe), "avg_launch_us": a["avg_launch_us"],
            "bytes_per_launch": a["bytes_per_launch"], "timed_launches": a["timed_launches"],
            "busy_launches": a["busy_launches"], "sample_every": every,
            "note": note or ("achieved = algorithmic bytes / HIP-event duration, summed over "
                             "the timed launches that did work")}


def torch_from(a, dev):
    import torch
    return torch.from_numpy(a).to(dev)


# ---------------------------------------------------------------------------------------
# batch512: the default line
# ---------------------------------------------------------------------------------------

def build_batch_systems(gsk, problems, dev, specs, keep_host=()):
    """Upload each system unscaled: CSR (kept for the one-at-a-time path) and 5/7-point
    planes (what the engine scales and solves). Host copies of the systems whose index is in
    keep_host are returned too (the CPU baseline's sample)."""
    systems, host = [], {}
    keep = set(keep_host)
    t0 = time.perf_counter()
    for i, sp in enumerate(specs):
        P = problems.batch_system(sp)
        A = gsk.CsrMatrix.from_problem(P, dev)
        d = list(P.dims) + [1] * (3 - len(P.dims))
        S = gsk.stencil_from_csr(A, *d)
        b = torch_from(P.b, dev)
        systems.append({"A": A, "S": S, "b": b, "n": P.n, "grid": tuple(d), "dim": len(P.dims)})
        if i in keep:
            host[i] = P
        if (i + 1) % 64 == 0:
            log(f"built {i + 1}/{len(specs)} systems ({time.perf_counter() - t0:.1f}s)")
    return systems, host


def batch_cpu_baseline(host, tol, threads):
    """The oracle (GS(2), then Bi-CGSTAB to tol; plain sequential C) on the sampled systems,
    one system per host thread (ctypes releases the interpreter lock during each call).
    value = converged sampled systems / wall seconds of the pool."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle

    def one(P):
        vo, bo, _, _ = oracle.gs_scale(P, P.b, 2)
        S = P.copy()
        S.val, S.b = vo, bo
        return oracle.bicgstab(S, bo, tol=tol)

    items = sorted(host.items())
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        results = list(ex.map(lambda kv: one(kv[1]), items))
    wall = time.perf_counter() - t0
    infos = [info for _, info in results]
    per_system = {i: r for (i, _), r in zip(items, results)}
    conv = sum(1 for i in infos if i.status == oracle.CONVERGED)
    cpu = host_cpu()
    return {"value": round(conv / wall, 4), "unit": "solves/s", "cores": threads,
            "kind": "oracle",
            "sample": (f"{len(items)} systems of the batch (seeded sample, default_rng(1007)), "
                       f"each GS(2) + Bi-CGSTAB to {tol:g} by the sequential C oracle, one system "
                       f"per thread on {threads} host threads; value = converged sampled systems "
                       f"/ wall time ({wall:.1f} s)"),
            "converged": conv, "wall_s": round(wall, 2),
            "iterations": int(sum(i.iters for i in infos)),
            "host_cpu": cpu["model"], "host_nproc": cpu["nproc"],
            "host_cores_available": cpu["cores_available"]}, per_system


def batch_oracle_parity(per_system, infos, xs):
    """The engine's results on the oracle's sampled systems (full batch, the timed launch
    configuration) against the oracle's: equal statuses, iteration counts (relative
    difference), and solutions (largest difference over the largest entry of the oracle's x;
    two solutions to a relative residual of 1e-8 may differ by up to cond(A) x 1e-8)."""
    import numpy as np
    st_eq, rel_it, rel_x = 0, [], []
    for i, (xo, io) in per_system.items():
        ig = infos[i]
        st_eq += int(ig.status == io.status)
        rel_it.append(abs(ig.iters - io.iters) / max(io.iters, 1))
        xg = xs[i].cpu().numpy()
        rel_x.append(float(np.max(np.abs(xg - xo)) / max(float(np.max(np.abs(xo))), 1e-300)))
    rel_it, rel_x = np.array(rel_it), np.array(rel_x)
    return {"systems": len(per_system), "status_equal": st_eq,
            "iters_within_5pct": int(np.sum(rel_it <= 0.05)),
            "iters_rel_diff": {"median": round(float(np.median(rel_it)), 4),
                               "max": round(float(np.max(rel_it)), 4)},
            "x_rel_diff": {"median": float(f"{np.median(rel_x):.3g}"),
                           "max": float(f"{np.max(rel_x):.3g}")}}


def batch_iter_bytes(systems, infos, gmres, mixed):
    """Algorithmic bytes of the Krylov iterations of one batch (the per-row figures of the
    kernel-class table in gsk.h, stencil matrices of 5 or 7 planes)."""
    iter_bytes = 0.0
    for i, s in enumerate(systems):
        info, n = infos[i], s["n"]
        planes = 7 if s["dim"] == 3 else 5
        if gmres:
            # Arnoldi step j: A reads the inner matrix and columns 0..j (column j twice) and
            # writes w; B and C read columns 0..j and w and write w or u_{j+1}
            vb = 4.0 if mixed else 8.0
            mat = vb * planes * n
            steps, m = info.iters, 20
            full, last = divmod(steps, m)
            js = [j for j in range(m)] * full + list(range(last))
            iter_bytes += sum(mat + vb * n * (j + 2) + 2 * vb * n * (j + 3) for j in js)
        elif mixed:
            # FP32 planes and r~ r^ p v t, FP64 x: P M + 24 n, S M + 12 n, U 40 n
            mat = 4.0 * n * planes
            iter_bytes += info.iters * (2 * mat + 76.0 * n)
            if info.iters > 0:
                iter_bytes -= (8.0 * n * (1 + info.restarts)
                               + (20.0 * n if info.half_step else 0.0))
        else:
            # P M + 48 n, S M + 24 n, U 64 n; the first P after a start or restart moves 16 n
            # less, and a half-step exit skips 40 n of U
            mat = 8.0 * n * planes
            iter_bytes += info.iters * (2 * mat + 136.0 * n)
            if info.iters > 0:
                iter_bytes -= (16.0 * n * (1 + info.restarts)
                               + (40.0 * n if info.half_step else 0.0))
    return iter_bytes


def status_counts(infos):
    c = {}
    for info in infos.values():
        c[info.status_name] = c.get(info.status_name, 0) + 1
    return c


def measured_copy_peak(dev, mib=1024, reps=10):
    """Achievable HBM bandwidth on this device, measured beside the roofline's published peak:
    a device-to-device copy of `mib` MiB (torch's copy kernel), best of `reps`, counting the
    bytes read and written."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del src, dst
    gbs = 2 * n * 8 / (best * 1e-3) / 1e9
    return {"GBs": round(gbs, 1), "frac_of_8TBs": round(gbs / HBM_PEAK_GBS, 4),
            "kernel": f"device-to-device copy of {mib} MiB (read + written bytes), best of {reps}"}


def device_info(dev):
    """What the runtime reports for the device the line was measured on (compute units, wave
    size, memory, L2), beside the published figures the roofline uses."""
    import torch
    pr = torch.cuda.get_device_properties(dev)
    return {"name": pr.name, "arch": getattr(pr, "gcnArchName", ""),
            "compute_units": pr.multi_processor_count, "wave_size": pr.warp_size,
            "hbm_GiB": round(pr.total_memory / 2 ** 30, 1),
            "l2_cache_bytes": getattr(pr, "L2_cache_size", None),
            "lds_bytes_per_workgroup": getattr(pr, "shared_memory_per_block", None)}


def bench_batch(args, gsk, problems, dev):
    """batch512: a batch of independent GS(2) + Bi-CGSTAB (or GMRES(20)) solves, tol 1e-8, run
    by the engine with every chunk replayed from a HIP graph."""
    import numpy as np
    import torch
    gmres = args.batch_method == "gmres"
    mixed = args.precision == "mixed"
    tol = 1e-8
    specs = problems.batch_specs(args.batch_count)
    want_cpu = not args.no_cpu_baseline and not gmres and not mixed
    sample = []
    if want_cpu:
        k = min(args.cpu_sample_systems, len(specs))
        sample = sorted(int(i) for i in np.random.default_rng(1007).choice(len(specs), k,
                                                                            replace=False))
    acc_sample = []
    if mixed and not gmres:
        # mixed results against the FP64 oracle's solutions: the 12 smallest systems of a
        # seeded sample of 48 (the oracle solves them in seconds)
        pool = np.random.default_rng(1008).choice(len(specs), 48, replace=False)
        acc_sample = sorted(sorted((int(i) for i in pool),
                                   key=lambda i: int(np.prod(specs[i]["dims"])))[:12])
        sample = sorted(set(sample) | set(acc_sample))
    systems, host = build_batch_systems(gsk, problems, dev, specs, keep_host=sample)
    unit = 512 if mixed else 256
    tuned = None
    check_every, tile_units, class_shapes = 8, 0, None
    if args.class_shapes and not gmres and not mixed:
        class_shapes = dict(kv.split("=") for kv in args.class_shapes.split(","))
        check_every = args.chunk or 16
        tuned = {"engine": "FP64 Bi-CGSTAB: launch shapes per size class given on the command "
                           "line", "class_shapes": class_shapes, "chunk": check_every}
    elif args.tile_units or args.chunk:
        tile_units, check_every = args.tile_units or 1, args.chunk or 8
    elif not gmres and not args.no_tune:
        # launch shapes and chunk length measured on the batch, before (and outside) the timing
        from paper_0812_2769_amd import tune
        t0 = time.perf_counter()
        if mixed:
            t = tune.tune_mixed_chunk(systems, device=dev, maxit=48)
            check_every = t["chunk"]
            tuned = {"engine": "mixed Bi-CGSTAB: two tiles per workgroup (FP32 data), chunk "
                               "length measured",
                     "chunk": check_every, "iterations_each": t["maxit"],
                     "chunk_seconds": {str(k): round(v, 4)
                                       for k, v in t["chunk_seconds"].items()}}
        else:
            t = tune.tune_classes(systems, device=dev, maxit=48)
            class_shapes, check_every = t["class_shapes"], t["chunk"]
            one = {name: min(tune.time_batch(systems, check_every, device=dev, tile_units=u,
                                             maxit=48) for _ in range(2))
                   for name, u in (("tile", 1), ("pair", 2))}
            tuned = {"engine": "FP64 Bi-CGSTAB: a launch shape per size class, each class "
                               "timed alone with every shape; then the chunk length",
                     "class_shapes": class_shapes, "chunk": check_every,
                     "iterations_each": t["maxit"],
                     "class_systems": t["class_systems"], "class_rows": t["class_rows"],
                     "class_seconds": {c: {k: round(v, 4) for k, v in d.items()}
                                       for c, d in t["class_seconds"].items()},
                     "chunk_seconds": {str(k): round(v, 4)
                                       for k, v in t["chunk_seconds"].items()},
                     "whole_batch_seconds": {
                         "per_class": round(t["chunk_seconds"][check_every], 4),
                         "one_shape_tile": round(one["tile"], 4),
                         "one_shape_pair": round(one["pair"], 4)}}
        tuned["tuning_s"] = round(time.perf_counter() - t0, 1)
        log(f"engine tuned: {tuned}")
    elif gmres:
        tuned = {"engine": f"GMRES(20) {'mixed' if mixed else 'FP64'}: shape fixed by the "
                           "single solver's partial sums (one tile per workgroup for FP64, "
                           "two for FP32 data); a chunk is one restart cycle"}
    if tile_units:
        unit = 256 * tile_units
    if class_shapes:
        unit = 512
    rows = sum((s["n"] + unit - 1) // unit * unit for s in systems)
    eng = gsk.Engine(rows, len(systems), check_every=check_every, graph=True, device=dev,
                     method=args.batch_method, m=20, precision="mixed" if mixed else "fp64",
                     tile_units=tile_units, class_shapes=class_shapes)
    solver = (f"GMRES(20) {'mixed precision' if mixed else 'FP64'}" if gmres
              else f"Bi-CGSTAB {'mixed precision' if mixed else 'FP64'}")
    xbuf = torch.zeros(sum(s["n"] for s in systems), dtype=torch.float64, device=dev)
    offs = [0]
    for s in systems:
        offs.append(offs[-1] + s["n"])
    xs = [xbuf[offs[i]:offs[i + 1]] for i in range(len(systems))]

    def step():
        xbuf.zero_()
        t0 = time.perf_counter()
        for i, s in enumerate(systems):
            assert eng.submit_gs(s["S"], s["b"], xs[i], p=2, tol=tol, tag=i)
        lat, infos = {}, {}
        while len(infos) < len(systems):
            eng.run(1)
            for tag, info in eng.poll():
                infos[tag] = info
                lat[tag] = time.perf_counter() - t0
        return lat, infos

    for i in range(args.warmup):
        step()
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    probe = args.probe or ("none" if gmres or mixed else "batch_p")
    if probe != "none":
        gsk.probe_begin(probe, args.probe_every)
    lats, infos = [], {}
    converged = 0
    t_start = time.perf_counter()
    for i in range(args.steps):
        lat, infos = step()
        lats.extend(lat.values())
        converged += sum(1 for v in infos.values() if v.status == gsk.CONVERGED)
        log(f"step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    pr = gsk.probe_end() if probe != "none" else None
    its = [infos[k].iters for k in infos]
    iter_bytes = batch_iter_bytes(systems, infos, gmres, mixed)
    row_iters = sum(infos[i].iters * s["n"] for i, s in enumerate(systems))
    not_conv = {str(k): {"status": v.status_name, "iters": v.iters,
                         "relres_true": v.relres_true}
                for k, v in sorted(infos.items()) if v.status != gsk.CONVERGED}
    if not_conv:
        log(f"WARNING {len(not_conv)} systems did not converge")
    out = {
        "metric": METRIC,
        "value": round(converged / elapsed, 3),
        "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 storage, f64 arithmetic and refinement" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": f"batch of {len(systems)} systems, d in {{2,3}}, N in [32,96], "
                               f"box jump 10^U(2,6), convection U(0,30), seed 1004; GS(2) + "
                               f"{solver} in the batch engine (HIP-graph chunks of "
                               f"{'one cycle' if gmres else f'{check_every} iterations'}), "
                               f"tol 1e-8",
                   "rows": sum(s["n"] for s in systems), "systems": len(systems),
                   "dims_3d": sum(1 for s in systems if s["dim"] == 3), "tol": tol,
                   "precision": args.precision, "method": args.batch_method},
        "solves_per_step": len(systems),
        "converged_per_step": converged / args.steps,
        "status": status_counts(infos),
        "fp64_continuations": (sum(1 for v in infos.values() if v.fp64_from > 0)
                               if mixed and not gmres else None),
        "not_converged": not_conv,
        "latency_p50_ms": round(1e3 * pct(lats, 0.5), 3),
        "latency_p99_ms": round(1e3 * pct(lats, 0.99), 3),
        "latency_note": "per system, from the batch's submission to the system's retirement",
        "iterations": {"total": int(sum(its)), "max": int(max(its)), "median": pct(its, 0.5),
                       "row_iterations": int(row_iters),
                       "per_s": round(sum(its) * args.steps / elapsed, 1)},
        "iteration_bandwidth": {
            "GB": round(iter_bytes / 1e9, 3),
            "GBs": round(iter_bytes / 1e9 / (elapsed / args.steps), 1),
            "frac_of_8TBs": round(iter_bytes / 1e9 / (elapsed / args.steps) / 8000.0, 4),
            "note": "algorithmic bytes of every Krylov iteration (Arnoldi step) of a step / "
                    "whole step time (GS, residual and finalize launches, host polls "
                    "included)"},
        "engine_tuning": tuned,
        "measured_copy_peak": measured_copy_peak(dev),
        "device": device_info(dev),
        "roofline": None, "cpu_baseline": None,
    }
    a = achieved(pr)
    if a is not None:
        traffic = (traffic_for(probe, None, "stencil", a["bytes_per_launch"])
                   if not gmres and not mixed else None)
        out["roofline"] = roofline_of(
            a, probe, args.probe_every, traffic=traffic,
            note=("achieved = algorithmic bytes of the timed launches (per running system at "
                  "that stage, the kernel-class table in gsk.h) / their HIP-event durations; "
                  "every k-th chunk of the timed steps runs without its graph and times each "
                  "launch of the class; traffic = the counter-measured ratio of HBM bytes to "
                  "algorithmic bytes of this class (FETCH_SIZE x 2.000 + WRITE_SIZE, full-batch "
                  "launches) times bytes_per_launch, null once the kernel sources change"))
    eng.close()
    if out["roofline"] is not None and probe == "batch_p":
        # the same 13-stream mix (7 planes, r, p, v, r^ read; p, v written) without gathers,
        # engine lookups or tails: what a kernel with P's mix can reach on this device
        c = gsk.stream_mix(11, 2, 40_000_000, reps=10, device=dev)
        out["stream_ceiling"] = {
            "mix": "P's arrays: 11 read, 2 written, one row per thread, 8-byte loads, tile "
                   "reductions, no gathers (gsk_stream_mix_ms, 40 M rows, best of 10)",
            "GBs": round(c["GBs"], 1), "frac_of_8TBs": round(c["GBs"] / HBM_PEAK_GBS, 4),
            "kernel_frac_of_ceiling": round(out["roofline"]["achieved"] / c["GBs"], 4)}
    if acc_sample:
        import oracle
        errs = {}
        for i in acc_sample:
            P = host[i]
            vo, bo, _, _ = oracle.gs_scale(P, P.b, 2)
            S = P.copy()
            S.val, S.b = vo, bo
            x64, i64 = oracle.bicgstab(S, bo, tol=tol)
            xg = xs[i].cpu().numpy()
            errs[str(i)] = {"n": P.n, "x_rel_error_vs_fp64_oracle":
                            float(np.linalg.norm(xg - x64) / np.linalg.norm(x64)),
                            "oracle_status": i64.status_name,
                            "relres_true_mixed": infos[i].relres_true}
        ev = [e["x_rel_error_vs_fp64_oracle"] for e in errs.values()]
        out["accuracy_vs_fp64_oracle"] = {
            "systems": errs, "max": max(ev), "median": pct(ev, 0.5),
            "note": "x of the mixed engine against orc_bicgstab's x (FP64, same tol) on the 12 "
                    "smallest of 48 seeded systems; two solutions with residual below tol "
                    "differ by up to about cond(A) tol"}
    if not args.no_solo and not (mixed and not gmres):
        # the same solves one at a time: gsk_gs_scale + packing + the single solver per system
        log("timing the one-at-a-time path")
        ws_gs = gsk.workspace(gsk.METHOD_GS, 1, 0, dev)
        nmax = max(s["n"] for s in systems)
        meth = (gsk.METHOD_GMRES_MIXED if mixed else gsk.METHOD_GMRES) if gmres \
            else gsk.METHOD_BICGSTAB
        ws_so = gsk.workspace(meth, nmax, 20 if gmres else 0, dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        same = True
        conv_solo = 0
        for i, s in enumerate(systems):
            As, bs, _, _ = gsk.gs_scale(s["A"], s["b"], 2, want_norms=False, ws=ws_gs)
            M = gsk.stencil_from_csr(As, *s["grid"], ws=ws_gs)
            ws = ws_so[: gsk.workspace_bytes_for(M, meth, 20 if gmres else 0)]
            if gmres:
                x, info = (gsk.gmres_mixed if mixed else gsk.gmres)(M, bs, m=20, tol=tol, ws=ws)
            else:
                x, info = gsk.bicgstab(M, bs, tol=tol, ws=ws)
            conv_solo += info.status == gsk.CONVERGED
            same = same and info == infos[i] and bool(torch.equal(x, xs[i]))
        torch.cuda.synchronize()
        t_solo = time.perf_counter() - t0
        out["one_at_a_time"] = {"converged_per_s": round(conv_solo / t_solo, 3),
                                "seconds": round(t_solo, 3),
                                "results_bitwise_equal_to_batch": same}
        del ws_so
    if want_cpu:
        threads = cpu_threads()
        log(f"timing the CPU oracle on {len(host)} sampled systems, {threads} threads")
        out["cpu_baseline"], per_system = batch_cpu_baseline(host, tol, threads)
        out["oracle_parity"] = batch_oracle_parity(per_system, infos, xs)
    if not args.no_extras and not gmres and not mixed:
        del systems, xs, xbuf
        torch.cuda.empty_cache()
        log("extras: 80^3 slabs")
        ex = {"slabs80": extra_slabs80(gsk, problems, dev)}
        log("extras: 64^2 square jump")
        ex["square64"] = extra_square64(gsk, problems, dev, cpu=want_cpu)
        torch.cuda.empty_cache()
        log("extras: 160^3 checkerboard")
        ex["checker160"] = extra_checker160(gsk, problems, dev)
        out["extras"] = ex
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------------------------------
# one large system at a time: slabs80, checker160
# ---------------------------------------------------------------------------------------

class Single:
    """One system with preallocated outputs and workspaces: solve(p, method, precision) runs
    GS(p) out of place from the unscaled CSR matrix, packs the scaled matrix into stencil
    planes (stencil operator) and runs the solver; the matrix stays resident in HBM."""

    def __init__(self, gsk, P, dev, operator="stencil", m=30, mixed=False):
        import torch
        self.gsk, self.P, self.dev = gsk, P, dev
        self.grid = P.dims[0]
        self.A = gsk.CsrMatrix.from_problem(P, dev)
        self.b = torch.from_numpy(P.b).to(dev)
        n = self.n = P.n
        self.val_s = torch.empty_like(self.A.val)
        self.b_s = torch.empty_like(self.b)
        self.weights = torch.empty(n, dtype=torch.float64, device=dev)
        self.x = torch.empty(n, dtype=torch.float64, device=dev)
        self.ws_gs = gsk.workspace(gsk.METHOD_GS, n, 0, dev)
        self.m = m
        self.ws_gm = gsk.workspace(gsk.METHOD_GMRES, n, m, dev)
        self.ws_mx = gsk.workspace(gsk.METHOD_GMRES_MIXED, n, m, dev) if mixed else None
        self.ws_bi = gsk.workspace(gsk.METHOD_BICGSTAB, n, 0, dev)
        self.As = self.A.with_values(self.val_s)
        self.stencil = operator == "stencil"
        if self.stencil:
            self.coef = torch.empty(7 * n, dtype=torch.float64, device=dev)
            self.Ss = gsk.StencilMatrix(self.grid, self.grid, self.grid, self.coef)
        self.M = self.Ss if self.stencil else self.As

    def gs(self, p):
        self.gsk.gs_scale_into(self.A, self.b, p, self.val_s, self.b_s, self.weights,
                               ws=self.ws_gs)
        if self.stencil:
            self.gsk.stencil_from_csr(self.As, self.grid, self.grid, self.grid, out=self.coef,
                                      ws=self.ws_gs)

    def solve(self, p, method, precision="fp64", tol=1e-8, maxit=None):
        gsk = self.gsk
        self.gs(p)
        w = None if p == 2 else self.weights
        if method == "bicgstab":
            return gsk.bicgstab(self.M, self.b_s, tol=tol, maxit=maxit, stop_weights=w,
                                ws=self.ws_bi, x_out=self.x)[1]
        if precision == "mixed":
            return gsk.gmres_mixed(self.M, self.b_s, m=self.m, tol=tol, maxit=maxit,
                                   stop_weights=w, ws=self.ws_mx, x_out=self.x)[1]
        return gsk.gmres(self.M, self.b_s, m=self.m, tol=tol, maxit=maxit, stop_weights=w,
                         ws=self.ws_gm, x_out=self.x)[1]


def vkey(v):
    return f"gs{v[0]}_{v[1]}" + ("_mixed" if v[2] == "mixed" else "")


def run_variants(S, variants, steps, warmup, tol, maxit=None, probe="none", every=4):
    """Runs the variants (p, method, precision) `steps` times after `warmup` untimed rounds.
    Returns (elapsed, latencies per variant, last infos, probe result)."""
    import torch
    gsk = S.gsk
    lat = {vkey(v): [] for v in variants}
    infos = {}
    for i in range(warmup):
        for v in variants:
            S.solve(v[0], v[1], v[2], tol, maxit)
        log(f"warmup {i + 1}/{warmup} done")
    torch.cuda.synchronize()
    if probe != "none":
        gsk.probe_begin(probe, every)
    t_start = time.perf_counter()
    for i in range(steps):
        for v in variants:
            t = time.perf_counter()
            infos[vkey(v)] = S.solve(v[0], v[1], v[2], tol, maxit)
            lat[vkey(v)].append(time.perf_counter() - t)
        log(f"step {i + 1}/{steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    pr = gsk.probe_end() if probe != "none" else None
    return elapsed, lat, infos, pr


def cpu_baseline_single(P, gpu_iters, sample_iters, variants, tol):
    """Time the oracle (single thread) on a bounded sample of the step: GS(p) in full and
    `sample_iters` iterations of each solver; scale to one full step with the iteration
    counts of the GPU run (the same algorithm takes about the same number of iterations)."""
    import oracle
    t_total = 0.0
    detail = {}
    for v in variants:
        p, method, precision = v
        t0 = time.perf_counter()
        vo, bo, nrm, w = oracle.gs_scale(P, P.b, p)
        t_gs = time.perf_counter() - t0
        S = P.copy()
        S.val, S.b = vo, bo
        W = None if p == 2 else w
        t0 = time.perf_counter()
        if method == "bicgstab":
            _, info = oracle.bicgstab(S, bo, tol=tol, weights=W, maxit=sample_iters)
        elif precision == "mixed":
            _, info = oracle.gmres_ir(S, bo, m=30, tol=tol, weights=W, maxit=sample_iters)
        else:
            _, info = oracle.gmres(S, bo, m=30, tol=tol, weights=W, maxit=sample_iters)
        t_it = (time.perf_counter() - t0) / max(info.iters, 1)
        est = t_gs + t_it * gpu_iters[vkey(v)]
        detail[vkey(v)] = {"gs_s": round(t_gs, 4), "s_per_iter": round(t_it, 5),
                           "sampled_iters": info.iters, "est_solve_s": round(est, 3)}
        t_total += est
    cpu = host_cpu()
    return {"value": round(len(variants) / t_total, 4), "unit": "solves/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"GS(p) in full plus the first {sample_iters} iterations of each of the "
                       f"{len(variants)} solves, single-threaded C oracle; seconds/iteration "
                       f"scaled by the GPU run's iteration counts"),
            "host_cpu": cpu["model"], "host_nproc": cpu["nproc"], "per_variant": detail}


def per_variant_of(lat, infos):
    return {k: {"iters": infos[k].iters, "status": infos[k].status_name,
                "relres_true": infos[k].relres_true,
                "p50_ms": round(1e3 * pct(lat[k], 0.5), 3),
                "p99_ms": round(1e3 * pct(lat[k], 0.99), 3)} for k in lat}


def bench_slabs80(args, gsk, problems, dev):
    """slabs80: the 80^3 system's four solves (GS(2)/GS(1) x Bi-CGSTAB/GMRES(30)) to 1e-10."""
    import torch
    grid = args.grid or 80
    mixed = args.precision == "mixed"
    tol = 1e-10
    P = problems.slabs_3d(grid)
    log(f"generated {P.name} n={P.n} nnz={P.nnz}")
    S = Single(gsk, P, dev, args.operator, mixed=mixed)
    prec = "mixed" if mixed else "fp64"
    variants = [(2, "bicgstab", "fp64"), (2, "gmres30", prec), (1, "bicgstab", "fp64"),
                (1, "gmres30", prec)]
    probe = args.probe or "gmres_a"
    elapsed, lat, infos, pr = run_variants(S, variants, args.steps, args.warmup, tol,
                                           probe=probe, every=args.probe_every)
    converged = sum(1 for k in infos if infos[k].status == gsk.CONVERGED) * args.steps
    accuracy = None
    if mixed:
        # every mixed GMRES result against the FP64 solver on the same scaled system
        accuracy = {}
        ws64 = gsk.workspace(gsk.METHOD_GMRES, P.n, 30, dev)
        for v in variants:
            if v[1] != "gmres30":
                continue
            im = S.solve(v[0], v[1], "mixed", tol)
            xm = S.x.clone()
            w = None if v[0] == 2 else S.weights
            x64, i64 = gsk.gmres(S.M, S.b_s, m=30, tol=tol, stop_weights=w, ws=ws64)
            err = (torch.linalg.vector_norm(xm - x64) / torch.linalg.vector_norm(x64)).item()
            accuracy[vkey(v)] = {
                "x_rel_error_vs_fp64_gpu": err, "relres_true_mixed": im.relres_true,
                "relres_true_fp64": i64.relres_true, "steps_mixed": im.iters,
                "steps_fp64": i64.iters}
        del ws64
    kernels = {}
    if not args.no_kernel_table:
        for cls in gsk.SOLVER_KCLASSES:
            gsk.probe_begin(cls)
            for v in variants:
                S.solve(v[0], v[1], v[2], tol)
            kernels[cls] = achieved(gsk.probe_end())
        # the product alone (gsk_spmv) on the GS(2)-scaled matrix: CSR, and the stencil planes
        # when they are the operator; algorithmic bytes = matrix + x once + y
        S.gs(2)
        n = P.n
        products = [("spmv_csr", S.As, 12.0 * P.nnz + 4.0 * (n + 1) + 16.0 * n)]
        if S.stencil:
            products.append(("spmv_stencil", S.Ss, 56.0 * n + 16.0 * n))
        xs, ys = S.b_s.clone(), torch.empty_like(S.b_s)
        for name, Mx, nbytes in products:
            for _ in range(3):
                gsk.spmv(Mx, xs, out=ys)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(50):
                gsk.spmv(Mx, xs, out=ys)
            e1.record()
            e1.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / 50
            kernels[name] = {"achieved_GBs": round(nbytes / us / 1e3, 1),
                             "avg_launch_us": round(us, 3), "bytes_per_launch": int(nbytes),
                             "launches": 50, "note": "50 launches back to back, events around "
                                                     "all of them"}
    for key, info in infos.items():
        if info.status != gsk.CONVERGED:
            log(f"WARNING {key} ended {info.status_name} at relres {info.relres_true:.2e}")
    all_lat = [v for k in lat for v in lat[k]]
    out = {
        "metric": METRIC,
        "value": round(converged / elapsed, 4), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64; GMRES f32 storage with f64 refinement" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": f"{grid}^3 7-point convection-diffusion, 8 random slabs "
                               f"(seed 1002), FP64 CSR; GS(1|2) x (Bi-CGSTAB | GMRES(30)), "
                               f"tol 1e-10",
                   "n": P.n, "nnz": P.nnz, "solves_per_step": len(variants), "tol": tol,
                   "operator": args.operator, "precision": args.precision},
        "iterations_per_s": round(sum(i.iters for i in infos.values()) * args.steps / elapsed,
                                  1),
        "latency_p50_ms": round(1e3 * pct(all_lat, 0.5), 3),
        "latency_p99_ms": round(1e3 * pct(all_lat, 0.99), 3),
        "per_variant": per_variant_of(lat, infos),
        "accuracy_vs_fp64": accuracy,
        "roofline": None, "cpu_baseline": None, "kernels": kernels,
        "cache_note": ("the GMRES(30) working set (~185 MB) fits in the 256 MB Infinity Cache: "
                       "achieved bandwidth here is fabric (HBM + cache) bandwidth"),
    }
    a = achieved(pr)
    if a is not None:
        out["roofline"] = roofline_of(a, probe, args.probe_every,
                                      traffic_for(probe, grid, args.operator,
                                                  a["bytes_per_launch"]) if not mixed
                                      else None)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline_single(P, {k: infos[k].iters for k in infos},
                                                  args.cpu_sample_iters, variants, tol)
    print(json.dumps(out), flush=True)


def bench_checker160(args, gsk, problems, dev):
    """checker160: GS(2) + Bi-CGSTAB to 1e-8 (value = its converged solves/s), and GMRES(30)
    in FP64 and mixed precision to the 10,000-step cap (or --checker-steps), with the relative
    residual reached and Arnoldi steps/s; k_gmres_a timed with HIP events."""
    grid = args.grid or 160
    tol = 1e-8
    maxit = args.checker_steps or None
    P = problems.checkerboard_3d(grid)
    log(f"generated {P.name} n={P.n} nnz={P.nnz}")
    S = Single(gsk, P, dev, args.operator, mixed=True)
    probe = args.probe or "gmres_a"
    vb = [(2, "bicgstab", "fp64")]
    vg = [(2, "gmres30", "fp64"), (2, "gmres30", "mixed")]
    el_b, lat_b, inf_b, _ = run_variants(S, vb, args.steps, args.warmup, tol)
    el_g, lat_g, inf_g, pr = run_variants(S, vg, args.steps, min(args.warmup, 1), tol, maxit,
                                          probe=probe, every=args.probe_every)
    conv_b = sum(1 for k in inf_b if inf_b[k].status == gsk.CONVERGED) * args.steps
    gm = {}
    for k, info in inf_g.items():
        t = pct(lat_g[k], 0.5)
        gm[k] = {"steps": info.iters, "status": info.status_name,
                 "relres_true": info.relres_true, "p50_s": round(t, 3),
                 "arnoldi_steps_per_s": round(info.iters / t, 1)}
    lat = dict(lat_b)
    lat.update(lat_g)
    infos = dict(inf_b)
    infos.update(inf_g)
    out = {
        "metric": METRIC,
        "value": round(conv_b / el_b, 4), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * (el_b + el_g) / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{grid}^3 7-point, 16^3-block checkerboard a in {{1, 1e4}} "
                               f"(seed 1003), FP64 CSR; GS(2) + Bi-CGSTAB to 1e-8 (value); "
                               f"GS(2) + GMRES(30) FP64 and FP32-storage/FP64-refinement to "
                               f"{maxit or 10000} steps",
                   "n": P.n, "nnz": P.nnz, "tol": tol, "operator": args.operator},
        "value_note": "converged GS(2) + Bi-CGSTAB solves per second; restarted GMRES(30) does "
                      "not reach 1e-8 within the 10,000-step cap on this system (its relative "
                      "residual is listed)",
        "latency_p50_ms": round(1e3 * pct(lat_b["gs2_bicgstab"], 0.5), 3),
        "latency_p99_ms": round(1e3 * pct(lat_b["gs2_bicgstab"], 0.99), 3),
        "per_variant": per_variant_of(lat, infos),
        "gmres": gm,
        "roofline": None, "cpu_baseline": None,
    }
    a = achieved(pr)
    if a is not None:
        out["roofline"] = roofline_of(a, probe, args.probe_every,
                                      note="FP64 and mixed GMRES(30) launches of the class "
                                           "together")
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        its = {k: infos[k].iters for k in infos}
        out["cpu_baseline"] = cpu_baseline_single(P, its, 10, vb + vg, tol)
    print(json.dumps(out), flush=True)


def extra_slabs80(gsk, problems, dev):
    """The 80^3 slabs system's four solves to 1e-10, 3 timed rounds, k_gmres_a timed."""
    P = problems.slabs_3d(80)
    S = Single(gsk, P, dev, "stencil")
    variants = [(2, "bicgstab", "fp64"), (2, "gmres30", "fp64"), (1, "bicgstab", "fp64"),
                (1, "gmres30", "fp64")]
    steps = 3
    elapsed, lat, infos, pr = run_variants(S, variants, steps, 1, 1e-10, probe="gmres_a",
                                           every=4)
    conv = sum(1 for k in infos if infos[k].status == gsk.CONVERGED) * steps
    a = achieved(pr)
    return {"workload": "80^3 7-point, 8 random slabs (seed 1002); GS(1|2) x (Bi-CGSTAB | "
                        "GMRES(30)) FP64, tol 1e-10, stencil operator",
            "solves_per_s": round(conv / elapsed, 3), "steps": steps,
            "per_variant": per_variant_of(lat, infos),
            "k_gmres_a_fabric_GBs": a["achieved_GBs"] if a else None,
            "k_gmres_a_avg_launch_us": a["avg_launch_us"] if a else None,
            "note": "working set fits in the 256 MB Infinity Cache: fabric bandwidth, not an "
                    "HBM figure"}


def square64_cpu_baseline(P):
    """The oracle's time for the 64^2 solves (GS(2), then GMRES(20) to the step cap or
    Bi-CGSTAB to 1e-8), one solve each on one host thread."""
    import oracle
    out = {}
    for method in ("gmres20", "bicgstab"):
        t = time.perf_counter()
        vo, bo, _, _ = oracle.gs_scale(P, P.b, 2)
        S = P.copy()
        S.val, S.b = vo, bo
        if method == "gmres20":
            _, info = oracle.gmres(S, bo, m=20, tol=1e-8)
        else:
            _, info = oracle.bicgstab(S, bo, tol=1e-8)
        out[method] = {"seconds": round(time.perf_counter() - t, 3), "iters": info.iters,
                       "status": info.status_name}
    cpu = host_cpu()
    conv = out["bicgstab"]["status"] == "converged"
    return {"value": round(conv / out["bicgstab"]["seconds"], 2), "unit": "solves/s",
            "cores": 1, "kind": "oracle",
            "sample": "one GS(2) + Bi-CGSTAB solve to 1e-8 (value) and one GS(2) + GMRES(20) "
                      "solve to the step cap, sequential C oracle, one host thread",
            "per_method": out, "host_cpu": cpu["model"], "host_nproc": cpu["nproc"]}


def extra_square64(gsk, problems, dev, solves=30, gmres_solves=5, cpu=True):
    """The 64^2 square-jump system (4,096 unknowns) from the unscaled CSR matrix in HBM, scaled
    by GS(2) and packed into 5-point planes for each solve, one solve at a time, tol 1e-8:
    GMRES(20), which stagnates near 4.5e-4 on this system and runs to the 10,000-step cap
    (reported with the residual it reached), and Bi-CGSTAB, which converges. At this size a
    solve is bound by launch and reduction latency, not bandwidth: the figures are latency,
    steps/s and solves/s, beside the oracle's time for the same solves (cpu_baseline)."""
    import torch
    P = problems.square_jump_2d(64)
    N = P.dims[0]
    A = gsk.CsrMatrix.from_problem(P, dev)
    b = torch.from_numpy(P.b).to(dev)
    val_s, b_s = torch.empty_like(A.val), torch.empty_like(b)
    x = torch.empty_like(b)
    coef = torch.empty(5 * P.n, dtype=torch.float64, device=dev)
    As = A.with_values(val_s)
    S = gsk.StencilMatrix(N, N, 1, coef)
    ws_gs = gsk.workspace(gsk.METHOD_GS, P.n, 0, dev)
    ws_gm = gsk.workspace(gsk.METHOD_GMRES, P.n, 20, dev)
    ws_bi = gsk.workspace(gsk.METHOD_BICGSTAB, P.n, 0, dev)

    def solve(method):
        gsk.gs_scale_into(A, b, 2, val_s, b_s, ws=ws_gs)
        gsk.stencil_from_csr(As, N, N, 1, out=coef, ws=ws_gs)
        if method == "gmres20":
            return gsk.gmres(S, b_s, m=20, tol=1e-8, ws=ws_gm, x_out=x)[1]
        return gsk.bicgstab(S, b_s, tol=1e-8, ws=ws_bi, x_out=x)[1]

    out = {"workload": "64^2 5-point, a = 1e3 on the centred square, convection (10, 10); "
                       "GS(2) + GMRES(20) or Bi-CGSTAB, FP64, tol 1e-8, stencil operator",
           "note": "latency-bound: 4,096 rows are 16 tiles"}
    for method, count in (("gmres20", gmres_solves), ("bicgstab", solves)):
        for _ in range(2):
            solve(method)
        torch.cuda.synchronize()
        lat = []
        t0 = time.perf_counter()
        for _ in range(count):
            t = time.perf_counter()
            info = solve(method)
            lat.append(time.perf_counter() - t)
        elapsed = time.perf_counter() - t0
        out[method] = {"solves": count, "iters": info.iters, "status": info.status_name,
                       "relres_true": info.relres_true,
                       "converged_per_s": round(count * (info.status == gsk.CONVERGED)
                                                / elapsed, 2),
                       "iters_per_s": round(count * info.iters / elapsed, 1),
                       "p50_ms": round(1e3 * pct(lat, 0.5), 3),
                       "p99_ms": round(1e3 * pct(lat, 0.99), 3)}
    out["cpu_baseline"] = square64_cpu_baseline(P) if cpu else None
    return out


def extra_checker160(gsk, problems, dev):
    """The 160^3 checkerboard (HBM-resident): FP64 k_gmres_a over two GMRES(30) cycles, every
    launch timed; GS(2) + Bi-CGSTAB to 1e-8 timed once."""
    P = problems.checkerboard_3d(160)
    S = Single(gsk, P, dev, "stencil")
    _, _, _, pr = run_variants(S, [(2, "gmres30", "fp64")], 1, 1, 1e-8, maxit=60,
                               probe="gmres_a", every=1)
    a = achieved(pr)
    el, lat, infos, _ = run_variants(S, [(2, "bicgstab", "fp64")], 1, 1, 1e-8)
    info = infos["gs2_bicgstab"]
    return {"workload": "160^3 7-point, 16^3-block checkerboard a in {1, 1e4} (seed 1003), "
                        "stencil operator",
            "k_gmres_a_fp64": None if a is None else roofline_of(
                a, "gmres_a", 1, traffic=traffic_for("gmres_a", 160, "stencil",
                                                     a["bytes_per_launch"]),
                note="two GMRES(30) cycles (60 Arnoldi steps), every launch timed; HBM-resident "
                     "working set (1.2 GB); traffic = the counter-measured ratio of HBM to "
                     "algorithmic bytes of these launches times bytes_per_launch"),
            "bicgstab_to_1e-8": {"solves_per_s": round((info.status == gsk.CONVERGED) / el, 4),
                                 "seconds": round(el, 3), "iters": info.iters,
                                 "status": info.status_name,
                                 "relres_true": info.relres_true}}


# ---------------------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------------------

def bench_serve(args, gsk, problems, dev):
    """serving: Poisson arrivals of solves drawn from the batch recipe (a pool of systems
    drawn with seed 1005; each request picks one uniformly), a GMRES(20) / Bi-CGSTAB mix, tol
    1e-8, GS(2) per request, served with continuous batching and admission by free device
    memory (engines sized from it); one run per arrival rate. value = converged solves/s at
    the highest rate."""
    import numpy as np
    from paper_0812_2769_amd import serve
    rates = [float(r) for r in args.rates.split(",") if r]
    pool_specs = problems.batch_specs(args.serve_pool, seed=1005)
    pool, _ = build_batch_systems(gsk, problems, dev, pool_specs)
    nmax = max(s["n"] for s in pool)
    rng = np.random.default_rng(1006)
    srv = serve.Server(0, 256, check_every=8, graph=True, gmres_rows=nmax, m_max=20,
                       device=dev, gmres_lanes=args.gmres_lanes, gmres_mode=args.gmres_mode,
                       gmres_precision=args.gmres_precision, gmres_engine_systems=128,
                       tile_units=args.tile_units)
    log(f"engines sized from free device memory: {srv.sizing}")
    results = []
    for rate in rates:
        gaps = rng.exponential(1.0 / rate, size=args.serve_requests)
        arrivals = np.cumsum(gaps)
        picks = rng.integers(0, len(pool), size=args.serve_requests)
        kinds = rng.random(args.serve_requests) < args.gmres_share
        reqs = []
        for k in range(args.serve_requests):
            s = pool[int(picks[k])]
            reqs.append(serve.Request(tag=k, arrival=float(arrivals[k]), A=s["S"], b=s["b"],
                                      method="gmres" if kinds[k] else "bicgstab", m=20,
                                      tol=1e-8, csr=s["A"], grid=s["grid"]))
        deferred0 = srv.gate.deferred
        t0 = time.perf_counter()
        done = srv.serve(reqs)
        wall = time.perf_counter() - t0
        lat = [d.latency for d in done]
        lat_b = [d.latency for d in done if d.method == "bicgstab"]
        lat_g = [d.latency for d in done if d.method == "gmres"]
        span = max(d.finished for d in done) - min(d.arrival for d in done)
        conv = sum(1 for d in done if d.info.status == gsk.CONVERGED)
        conv_b = sum(1 for d in done if d.info.status == gsk.CONVERGED and d.method == "bicgstab")
        st = {}
        for d in done:
            key = f"{d.method}_{d.info.status_name}"
            st[key] = st.get(key, 0) + 1
        results.append({"rate": rate, "requests": len(done),
                        "converged_per_s": round(conv / span, 2),
                        "bicgstab_converged_per_s": round(conv_b / span, 2),
                        "completed_per_s": round(len(done) / span, 2),
                        "wall_s": round(wall, 3),
                        "latency_p50_ms": round(1e3 * pct(lat, 0.5), 2),
                        "latency_p99_ms": round(1e3 * pct(lat, 0.99), 2),
                        "bicgstab_p50_ms": round(1e3 * pct(lat_b, 0.5), 2) if lat_b else None,
                        "bicgstab_p99_ms": round(1e3 * pct(lat_b, 0.99), 2) if lat_b else None,
                        "gmres_p50_ms": round(1e3 * pct(lat_g, 0.5), 2) if lat_g else None,
                        "gmres_p99_ms": round(1e3 * pct(lat_g, 0.99), 2) if lat_g else None,
                        "converged": conv, "status": st,
                        "memory_deferrals": srv.gate.deferred - deferred0})
        log(f"rate {rate}: {results[-1]}")
    srv.close()
    best = results[-1]
    out = {
        "metric": "converged solves/s under Poisson arrivals, p50/p99 latency",
        "value": best["converged_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": len(rates), "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": ("f64; GMRES f32 storage with f64 refinement"
                  if args.gmres_mode == "engine" and args.gmres_precision == "mixed" else "f64"),
        "data": "synthetic",
        "config": {"workload": f"serving: Poisson arrivals at {args.rates} req/s, "
                               f"{args.serve_requests} requests per rate drawn from a pool of "
                               f"{args.serve_pool} batch-recipe systems (seed 1005), "
                               f"{args.gmres_share:.0%} GMRES(20), the rest Bi-CGSTAB, tol "
                               f"1e-8, GS(2) per request; admission by free device memory; "
                               f"Bi-CGSTAB in the batch engine, GMRES "
                               + (f"in a GMRES(20) engine ({args.gmres_precision})"
                                  if args.gmres_mode == "engine"
                                  else f"on {args.gmres_lanes} lanes")},
        "engine_sizing": srv.sizing,
        "latency_p50_ms": best["latency_p50_ms"], "latency_p99_ms": best["latency_p99_ms"],
        "rates": results, "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); sharding a solve "
              "over several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": n * 8, "bytes_written": n * 8,
                          "copies": 5}), flush=True)
        return

    from paper_0812_2769_amd import gsk, problems

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "batch512":
        return bench_batch(args, gsk, problems, dev)
    if args.workload == "serving":
        return bench_serve(args, gsk, problems, dev)
    if args.workload == "checker160":
        return bench_checker160(args, gsk, problems, dev)
    return bench_slabs80(args, gsk, problems, dev)


if __name__ == "__main__":
    main()
