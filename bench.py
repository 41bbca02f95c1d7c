"""Benchmark: GS(p) + Krylov solves on the 80^3 convection-diffusion system, one MI355X.

Workload (seeded, synthetic; generated on the host, uploaded before timing): 80^3 interior
grid, 7-point central differences in flux form, diffusion piecewise constant over 8 z-slabs
with values 10^U(0,6) (numpy default_rng(1002)), convection (20,-10,5), b = A u* with
u* = sin(pi x) sin(pi y) sin(pi z); n = 512,000, nnz = 3,545,600, FP64 CSR with int32 indices.

One step = the workload's four solves, each from the unscaled CSR matrix resident in HBM:
GS(p) (out of place), with --operator stencil (the default) the packing of the scaled CSR
matrix into 7-point coefficient planes, then the Krylov solve from x0 = 0 to a relative
residual below 1e-10 (measured on the GS(2)-scaled system), for p in {2, 1} and solver in
{Bi-CGSTAB, GMRES(30)}. `value` = solves per second over the timed steps.

Prints one JSON line. Also reports iterations/s, per-variant p50/p99 latency, the achieved
bandwidth of the dominant kernel against the HBM roofline, and the CPU oracle's rate on a
bounded sample of the same work.

Other modes (not the default line):
  --precision mixed   the GMRES(30) solves use gsk_gmres_mixed (FP32 Arnoldi cycles, FP64
                      restarts) at the same tolerance; Bi-CGSTAB stays FP64.
  --workload checker160  the 160^3 checkerboard system (n = 4,096,000): GS(2) then
                      GMRES(30) bounded at 600 Arnoldi steps per solve (restarted GMRES(30) does
                      not reach the workload's 1e-8 within the 10,000-step cap); `value` is
                      Arnoldi steps per second.
  --workload batch512    512 independent 2D/3D systems through the batch engine.
  --workload serving     Poisson arrivals through the solve server.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solves/s at 1e-8 rel. residual, Krylov HBM GB/s vs peak, p50/p99 latency"
HBM_PEAK_GBS = 8000.0
VARIANTS = [(2, "bicgstab"), (2, "gmres30"), (1, "bicgstab"), (1, "gmres30")]
KERNEL_NAMES = {"gmres_a": "k_gmres_a (matrix product + CGS2 pass-1 dots)",
                "gmres_b": "k_gmres_b (CGS2 pass-1 update + pass-2 dots)",
                "gmres_c": "k_gmres_c (CGS2 pass-2 update + norm)",
                "bicg_p": "k_bicg_p (p update + matrix product + dots)",
                "bicg_s": "k_bicg_s (s + matrix product + dots)",
                "bicg_u": "k_bicg_u (x, r update + dots)",
                "residual": "k_*_residual (true residual)",
                "gmres_x": "k_gmres_x (x += V y)"}
TOL = 1e-10
METRIC_CHECKER = "Arnoldi steps/s, GMRES(30) on the 160^3 checkerboard system"

# Fabric (HBM + Infinity Cache) bytes per working launch of a kernel class, from two
# rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE; FETCH_SIZE scaled by 2.000 and WRITE_SIZE by
# 1.000 from a plain 512 MiB copy), recorded with the hash of the kernel sources they were
# measured on. A source change makes the figure stale and it is reported as null.
TRAFFIC = {"gmres_a": {"bytes_per_launch": 96161325, "grid": 80, "operator": "stencil",
                       "sources_sha256_16": "ba7a51460425de28"}}
TRAFFIC_SOURCES = ["paper_0812_2769_amd/csrc/gmres.hip", "paper_0812_2769_amd/csrc/gmres_body.hpp",
                   "paper_0812_2769_amd/csrc/gsk_dev.hpp"]


def traffic_for(probe, grid, operator):
    import hashlib
    rec = TRAFFIC.get(probe)
    if rec is None or rec["grid"] != grid or rec.get("operator", "csr") != operator:
        return None
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return rec["bytes_per_launch"] if h.hexdigest()[:16] == rec["sources_sha256_16"] else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["slabs80", "checker160", "batch512", "serving"],
                    default="slabs80")
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
    ap.add_argument("--batch-method", choices=["bicgstab", "gmres"], default="bicgstab",
                    help="batch512: the engine's solver (GMRES(20) with --precision)")
    ap.add_argument("--batch-count", type=int, default=512,
                    help="batch512: systems per batch (default 512)")
    ap.add_argument("--no-solo", action="store_true",
                    help="batch512: skip the one-at-a-time comparison")
    ap.add_argument("--rates", default="50,200,1000,2000",
                    help="serving: Poisson arrival rates to sweep (requests/s)")
    ap.add_argument("--serve-requests", type=int, default=400,
                    help="serving: requests per rate")
    ap.add_argument("--gmres-share", type=float, default=0.2,
                    help="serving: fraction of GMRES(20) requests (the rest Bi-CGSTAB)")
    ap.add_argument("--grid", type=int, default=0,
                    help="N of the N^3 grid (default 80 for slabs80, 160 for checker160)")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64",
                    help="GMRES solves in FP64 (default) or mixed precision")
    ap.add_argument("--checker-steps", type=int, default=600,
                    help="Arnoldi steps per checker160 solve (default 600)")
    ap.add_argument("--operator", choices=["stencil", "csr"], default="stencil",
                    help="matrix form the solvers read: 7-point coefficient planes packed from "
                         "the scaled CSR matrix inside each solve (default), or the CSR matrix")
    ap.add_argument("--cpu-sample-iters", type=int, default=120,
                    help="iterations per solver the CPU oracle runs for its baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--probe", default="gmres_a",
                    help="kernel class timed with HIP events during the timed steps "
                         "('none' to time nothing)")
    ap.add_argument("--probe-every", type=int, default=4,
                    help="time every k-th launch of the probed class (default 4)")
    ap.add_argument("--no-kernel-table", action="store_true",
                    help="skip the extra untimed step per kernel class")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB MiB (reference for HBM "
                         "byte counters) and exit")
    return ap.parse_args()


def pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo = int(k)
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def cpu_baseline(P, gpu_iters, sample_iters, variants, tol, precision):
    """Time the oracle (single thread) on a bounded sample of the step: GS(p) in full and
    `sample_iters` iterations of each solver; scale to one full step with the iteration
    counts of the GPU run (the same algorithm takes about the same number of iterations)."""
    import oracle
    t_total = 0.0
    detail = {}
    for p, method in variants:
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
        key = f"gs{p}_{method}"
        est = t_gs + t_it * gpu_iters[key]
        detail[key] = {"gs_s": round(t_gs, 4), "s_per_iter": round(t_it, 5),
                       "sampled_iters": info.iters, "est_solve_s": round(est, 3)}
        t_total += est
    return {"value": round(len(variants) / t_total, 4), "unit": "solves/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"GS(p) in full plus the first {sample_iters} iterations of each of the "
                       f"{len(variants)} solves, single-threaded C oracle; seconds/iteration "
                       f"scaled by the GPU run's iteration counts"),
            "per_variant": detail}


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def build_batch_systems(gsk, problems, dev, specs):
    """Upload each system unscaled: CSR (kept for the one-at-a-time path) and 5/7-point
    planes (what the engine scales and solves)."""
    systems = []
    t0 = time.perf_counter()
    for i, sp in enumerate(specs):
        P = problems.batch_system(sp)
        A = gsk.CsrMatrix.from_problem(P, dev)
        d = list(P.dims) + [1] * (3 - len(P.dims))
        S = gsk.stencil_from_csr(A, *d)
        b = torch_from(P.b, dev)
        systems.append({"A": A, "S": S, "b": b, "n": P.n, "grid": tuple(d), "dim": len(P.dims)})
        if (i + 1) % 64 == 0:
            log(f"built {i + 1}/{len(specs)} systems ({time.perf_counter() - t0:.1f}s)")
    return systems


def torch_from(a, dev):
    import torch
    return torch.from_numpy(a).to(dev)


def bench_batch(args, gsk, problems, dev):
    """batch512: a batch of independent GS(2) + Bi-CGSTAB solves, tol 1e-8, run by the engine
    with every chunk replayed from a HIP graph. value = systems solved per second."""
    import torch
    specs = problems.batch_specs(args.batch_count)
    systems = build_batch_systems(gsk, problems, dev, specs)
    gmres = args.batch_method == "gmres"
    mixed = args.precision == "mixed"
    unit = 512 if mixed else 256
    rows = sum((s["n"] + unit - 1) // unit * unit for s in systems)
    tuned = None
    check_every, tile_units = 8, 0
    if args.tile_units or args.chunk:
        tile_units, check_every = args.tile_units or 1, args.chunk or 8
        unit = 256 * tile_units
        rows = sum((s["n"] + unit - 1) // unit * unit for s in systems)
    elif not gmres and not mixed and not args.no_tune:
        # launch shape and chunk length measured on a sample of the batch, before (and
        # outside) the timing
        from paper_0812_2769_amd import tune
        tuned = tune.tune_engine(systems, device=dev, maxit=48)
        tile_units, check_every = tuned["best"]
        unit = 256 * tile_units
        rows = sum((s["n"] + unit - 1) // unit * unit for s in systems)
        log(f"engine tuned on {tuned['sample']} systems x {tuned['maxit']} iterations: "
            f"{ {f'{u}x{k}': round(v, 4) for (u, k), v in tuned['seconds'].items()} } -> "
            f"{tile_units} tile(s) per workgroup, chunks of {check_every}")
    eng = gsk.Engine(rows, len(systems), check_every=check_every, graph=True, device=dev,
                     method=args.batch_method, m=20, precision="mixed" if mixed else "fp64",
                     tile_units=tile_units)
    solver = (f"GMRES(20) {'mixed precision' if mixed else 'FP64'}" if gmres
              else f"Bi-CGSTAB {'mixed precision' if mixed else 'FP64'}")
    xbuf = torch.zeros(sum(s["n"] for s in systems), dtype=torch.float64, device=dev)
    offs = [0]
    for s in systems:
        offs.append(offs[-1] + s["n"])
    xs = [xbuf[offs[i]:offs[i + 1]] for i in range(len(systems))]
    tol = 1e-8

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
    lats, infos = [], {}
    t_start = time.perf_counter()
    for i in range(args.steps):
        lat, infos = step()
        lats.extend(lat.values())
        log(f"step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    its = [infos[k].iters for k in infos]
    status = collections_count(infos)
    # Algorithmic bytes of the Bi-CGSTAB iterations of the last step (P, S and U launches, the
    # per-row figures of the kernel-class table in gsk.h for a stencil matrix of 5 or 7
    # planes): a full iteration moves 2 M + 136 n bytes with M = 8 n planes; the first P after
    # a start or restart moves 16 n less, and a half-step exit skips 40 n of U.
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
            mat = 8.0 * n * planes
            iter_bytes += info.iters * (2 * mat + 136.0 * n)
            if info.iters > 0:
                iter_bytes -= (16.0 * n * (1 + info.restarts)
                               + (40.0 * n if info.half_step else 0.0))
    row_iters = sum(infos[i].iters * s["n"] for i, s in enumerate(systems))
    out = {
        "metric": f"systems solved/s, batch of GS(2) + {solver}, tol 1e-8",
        "value": round(len(systems) * args.steps / elapsed, 3),
        "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"batch of {len(systems)} systems, d in {{2,3}}, N in [32,96], "
                               f"box jump 10^U(2,6), convection U(0,30); GS(2) + {solver} in "
                               f"the engine (HIP-graph chunks of "
                               f"{'one cycle' if gmres else f'{check_every} iterations'}), "
                               f"tol 1e-8",
                   "rows": sum(s["n"] for s in systems), "systems": len(systems),
                   "dims_3d": sum(1 for s in systems if s["dim"] == 3)},
        "latency_p50_ms": round(1e3 * pct(lats, 0.5), 3),
        "latency_p99_ms": round(1e3 * pct(lats, 0.99), 3),
        "iterations": {"total": int(sum(its)), "max": int(max(its)), "median": pct(its, 0.5),
                       "row_iterations": int(row_iters)},
        "iteration_bandwidth": {
            "GB": round(iter_bytes / 1e9, 3),
            "GBs": round(iter_bytes / 1e9 / (elapsed / args.steps), 1),
            "frac_of_8TBs": round(iter_bytes / 1e9 / (elapsed / args.steps) / 8000.0, 4),
            "note": "algorithmic bytes of every Krylov iteration (Arnoldi step) of a step / "
                    "whole step time (GS, residual and finalize launches, host polls "
                    "included)"},
        "status": status,
        "engine_tuning": None if tuned is None else {
            "tiles_per_workgroup": tuned["best"][0], "chunk": tuned["best"][1],
            "sample_systems": tuned["sample"], "iterations_each": tuned["maxit"],
            "seconds": {f"{u}x{k}": round(v, 4) for (u, k), v in tuned["seconds"].items()}},
        "roofline": None, "cpu_baseline": None,
    }
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
        for i, s in enumerate(systems):
            As, bs, _, _ = gsk.gs_scale(s["A"], s["b"], 2, want_norms=False, ws=ws_gs)
            M = gsk.stencil_from_csr(As, *s["grid"], ws=ws_gs)
            ws = ws_so[: gsk.workspace_bytes_for(M, meth, 20 if gmres else 0)]
            if gmres:
                x, info = (gsk.gmres_mixed if mixed else gsk.gmres)(M, bs, m=20, tol=tol, ws=ws)
            else:
                x, info = gsk.bicgstab(M, bs, tol=tol, ws=ws)
            same = same and info == infos[i] and bool(torch.equal(x, xs[i]))
        torch.cuda.synchronize()
        t_solo = time.perf_counter() - t0
        out["one_at_a_time"] = {"solves_per_s": round(len(systems) / t_solo, 3),
                                "seconds": round(t_solo, 3),
                                "results_bitwise_equal_to_batch": same}
    print(json.dumps(out), flush=True)


def collections_count(infos):
    c = {}
    for info in infos.values():
        c[info.status_name] = c.get(info.status_name, 0) + 1
    return c


def bench_serve(args, gsk, problems, dev):
    """serving: Poisson arrivals of solves drawn from the batch recipe (a pool of 64
    systems), a GMRES(20) / Bi-CGSTAB mix, tol 1e-8, served with continuous batching; one run
    per arrival rate. value = completed solves/s at the highest rate."""
    import numpy as np
    import torch
    from paper_0812_2769_amd import serve
    rates = [float(r) for r in args.rates.split(",") if r]
    pool_specs = problems.batch_specs(64, seed=1005)
    pool = build_batch_systems(gsk, problems, dev, pool_specs)
    nmax = max(s["n"] for s in pool)
    rng = np.random.default_rng(1006)
    # engine room for about 48 of the pool's systems at once
    unit = 256 * max(1, args.tile_units)
    rows = int(sum((s["n"] + unit - 1) // unit * unit for s in pool) * 0.75)
    srv = serve.Server(rows, 256, check_every=8, graph=True, gmres_rows=nmax, m_max=20,
                       device=dev, gmres_lanes=args.gmres_lanes, gmres_mode=args.gmres_mode,
                       gmres_precision=args.gmres_precision, gmres_engine_rows=rows,
                       gmres_engine_systems=128, tile_units=args.tile_units)
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
        t0 = time.perf_counter()
        done = srv.serve(reqs)
        wall = time.perf_counter() - t0
        lat = [d.latency for d in done]
        lat_b = [d.latency for d in done if d.method == "bicgstab"]
        lat_g = [d.latency for d in done if d.method == "gmres"]
        span = max(d.finished for d in done) - min(d.arrival for d in done)
        conv = sum(1 for d in done if d.info.status == gsk.CONVERGED)
        results.append({"rate": rate, "requests": len(done), "completed_per_s": round(len(done) / span, 2),
                        "wall_s": round(wall, 3),
                        "latency_p50_ms": round(1e3 * pct(lat, 0.5), 2),
                        "latency_p99_ms": round(1e3 * pct(lat, 0.99), 2),
                        "bicgstab_p50_ms": round(1e3 * pct(lat_b, 0.5), 2) if lat_b else None,
                        "gmres_p50_ms": round(1e3 * pct(lat_g, 0.5), 2) if lat_g else None,
                        "converged": conv})
        log(f"rate {rate}: {results[-1]}")
    srv.close()
    best = results[-1]
    out = {
        "metric": "completed solves/s under Poisson arrivals, p50/p99 latency",
        "value": best["completed_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": len(rates), "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": ("f64; GMRES f32 inner / f64 restarts"
                  if args.gmres_mode == "engine" and args.gmres_precision == "mixed" else "f64"),
        "data": "synthetic",
        "config": {"workload": f"serving: Poisson arrivals at {args.rates} req/s, "
                               f"{args.serve_requests} requests per rate from a pool of 64 "
                               f"batch-recipe systems, {args.gmres_share:.0%} GMRES(20), "
                               f"the rest Bi-CGSTAB, tol 1e-8, GS(2) per request; Bi-CGSTAB "
                               f"in the engine, GMRES "
                               + (f"in a GMRES(20) engine ({args.gmres_precision})"
                                  if args.gmres_mode == "engine"
                                  else f"on {args.gmres_lanes} lanes")},
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
    import numpy as np
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
    checker = args.workload == "checker160"
    grid = args.grid or (160 if checker else 80)
    variants = [(2, "gmres30")] if checker else VARIANTS
    tol = 1e-8 if checker else TOL
    maxit = args.checker_steps if checker else None
    t0 = time.perf_counter()
    P = problems.checkerboard_3d(grid) if checker else problems.slabs_3d(grid)
    print(f"bench: generated {P.name} n={P.n} nnz={P.nnz} in {time.perf_counter() - t0:.1f}s",
          file=sys.stderr, flush=True)
    A = gsk.CsrMatrix.from_problem(P, dev)
    b = torch.from_numpy(P.b).to(dev)
    n = P.n
    # Preallocated outputs and workspaces (outside the timed region)
    val_s = torch.empty_like(A.val)
    b_s = torch.empty_like(b)
    weights = torch.empty(n, dtype=torch.float64, device=dev)
    x = torch.empty(n, dtype=torch.float64, device=dev)
    ws_gs = gsk.workspace(gsk.METHOD_GS, n, 0, dev)
    mixed = args.precision == "mixed"
    ws_gm = gsk.workspace(gsk.METHOD_GMRES_MIXED if mixed else gsk.METHOD_GMRES, n, 30, dev)
    ws_bi = gsk.workspace(gsk.METHOD_BICGSTAB, n, 0, dev)
    As = A.with_values(val_s)
    c_A = A.c_struct()
    c_As = As.c_struct()
    import ctypes
    stream = torch.cuda.current_stream(dev).cuda_stream
    stencil = args.operator == "stencil"
    if stencil:
        coef = torch.empty(7 * n, dtype=torch.float64, device=dev)
        Ss = gsk.StencilMatrix(grid, grid, grid, coef)
    M = Ss if stencil else As

    def pack():
        rc = gsk.lib.gsk_stencil_from_csr(ctypes.byref(c_As), grid, grid, grid,
                                          coef.data_ptr(), ws_gs.data_ptr(), ws_gs.numel(),
                                          stream)
        if rc != 0:
            raise gsk.GskError(rc, gsk.lib.gsk_last_error().decode())

    def gs(p):
        rc = gsk.lib.gsk_gs_scale(ctypes.byref(c_A), b.data_ptr(), p, val_s.data_ptr(),
                                  b_s.data_ptr(), None, weights.data_ptr(), ws_gs.data_ptr(),
                                  ws_gs.numel(), stream)
        if rc != 0:
            raise gsk.GskError(rc, gsk.lib.gsk_last_error().decode())

    def solve(p, method):
        gs(p)
        if stencil:
            pack()
        w = None if p == 2 else weights
        if method == "bicgstab":
            return gsk.bicgstab(M, b_s, tol=tol, stop_weights=w, ws=ws_bi, x_out=x)[1]
        fn = gsk.gmres_mixed if mixed else gsk.gmres
        return fn(M, b_s, m=30, tol=tol, maxit=maxit, stop_weights=w, ws=ws_gm, x_out=x)[1]

    def step(lat, infos):
        for p, method in variants:
            t = time.perf_counter()
            info = solve(p, method)
            lat[f"gs{p}_{method}"].append(time.perf_counter() - t)
            infos[f"gs{p}_{method}"] = info

    lat = {f"gs{p}_{m}": [] for p, m in variants}
    infos = {}
    for i in range(args.warmup):
        step({k: [] for k in lat}, infos)
        print(f"bench: warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    if args.probe != "none":
        gsk.probe_begin(args.probe, args.probe_every)
    t_start = time.perf_counter()
    for i in range(args.steps):
        step(lat, infos)
        print(f"bench: step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    probe = gsk.probe_end() if args.probe != "none" else {"total_ms": 0, "busy_launches": 0}

    def achieved(pr):
        if pr["total_ms"] <= 0 or pr["busy_launches"] == 0:
            return None
        return {"achieved_GBs": round(pr["bytes"] / (pr["total_ms"] * 1e-3) / 1e9, 1),
                "avg_launch_us": round(1e3 * pr["total_ms"] / pr["busy_launches"], 3),
                "bytes_per_launch": round(pr["bytes"] / pr["busy_launches"]),
                "timed_launches": pr["launches"], "busy_launches": pr["busy_launches"]}

    # Mixed precision: every GMRES result against the FP64 solver on the same scaled system
    # (untimed). The FP64 path is the one the oracle parity tests pin.
    accuracy = None
    if mixed:
        accuracy = {}
        ws64 = gsk.workspace(gsk.METHOD_GMRES, n, 30, dev)
        for p, method in variants:
            if method != "gmres30":
                continue
            im = solve(p, method)
            xm = x.clone()
            w = None if p == 2 else weights
            x64, i64 = gsk.gmres(M, b_s, m=30, tol=tol, maxit=maxit, stop_weights=w, ws=ws64)
            err = (torch.linalg.vector_norm(xm - x64) / torch.linalg.vector_norm(x64)).item()
            accuracy[f"gs{p}_{method}"] = {
                "x_rel_error_vs_fp64": err, "relres_true_mixed": im.relres_true,
                "relres_true_fp64": i64.relres_true, "steps_mixed": im.iters,
                "steps_fp64": i64.iters}
        del ws64

    kernels = {}
    if not args.no_kernel_table:
        for cls in gsk.KCLASS:
            gsk.probe_begin(cls)
            step({k: [] for k in lat}, {})
            kernels[cls] = achieved(gsk.probe_end())
        # the product alone (gsk_spmv) on the GS(2)-scaled matrix: CSR, and the stencil planes
        # when they are the operator; algorithmic bytes = matrix + x once + y
        gs(2)
        products = [("spmv_csr", As, 12.0 * P.nnz + 4.0 * (n + 1) + 16.0 * n)]
        if stencil:
            pack()
            products.append(("spmv_stencil", Ss, 56.0 * n + 16.0 * n))
        xs, ys = b_s.clone(), torch.empty_like(b_s)
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
        if info.status != gsk.CONVERGED and not checker:
            print(f"bench: WARNING {key} ended {info.status_name} at relres "
                  f"{info.relres_true:.2e}", file=sys.stderr, flush=True)
    solves = len(variants) * args.steps
    iters_step = sum(i.iters for i in infos.values())
    per_variant = {k: {"iters": infos[k].iters, "status": infos[k].status_name,
                       "relres_true": infos[k].relres_true,
                       "p50_ms": round(1e3 * pct(lat[k], 0.5), 3),
                       "p99_ms": round(1e3 * pct(lat[k], 0.99), 3)} for k in lat}
    all_lat = [v for k in lat for v in lat[k]]
    out = {
        "metric": METRIC_CHECKER if checker else METRIC,
        "value": round((iters_step * args.steps if checker else solves) / elapsed, 4),
        "unit": "Arnoldi steps/s" if checker else "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 inner / f64 restarts" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": (
                       f"{grid}^3 7-point, 16^3-block checkerboard a in {{1, 1e4}}, "
                       f"FP64 CSR; GS(2) x GMRES(30) bounded at {args.checker_steps} steps" if checker else
                       f"{grid}^3 7-point convection-diffusion, 8 random slabs, FP64 "
                       f"CSR; GS(1|2) x (Bi-CGSTAB | GMRES(30)), tol 1e-10"),
                   "n": n, "nnz": P.nnz, "solves_per_step": len(variants), "tol": tol,
                   "operator": args.operator, "precision": args.precision},
        "iterations_per_s": round(iters_step * args.steps / elapsed, 1),
        "latency_p50_ms": round(1e3 * pct(all_lat, 0.5), 3),
        "latency_p99_ms": round(1e3 * pct(all_lat, 0.99), 3),
        "per_variant": per_variant,
        "accuracy_vs_fp64": accuracy,
        "roofline": None,
        "cpu_baseline": None,
        "kernels": kernels,
    }
    a = achieved(probe)
    if a is not None:
        out["roofline"] = {
            "bound": "hbm", "achieved": a["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(a["achieved_GBs"] / HBM_PEAK_GBS, 4),
            "traffic": (traffic_for(args.probe, grid, args.operator)
                        if not mixed and not checker else None),
            "kernel": KERNEL_NAMES.get(args.probe), "avg_launch_us": a["avg_launch_us"],
            "bytes_per_launch": a["bytes_per_launch"], "timed_launches": a["timed_launches"],
            "busy_launches": a["busy_launches"], "sample_every": args.probe_every,
            "note": ("achieved = algorithmic bytes / HIP-event duration, summed over the timed "
                     "launches that did work (every k-th launch of the class during the timed "
                     "steps)")}
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(P, {k: infos[k].iters for k in infos},
                                           args.cpu_sample_iters if not checker else 10, variants,
                                           tol, args.precision)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
