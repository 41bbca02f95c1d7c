"""Writes tests/golden/paper_tables_oracle.json: the oracle's results on the paper's tables that
are too slow to recompute inside the CPU test suite (up to 10,000 preconditioned GMRES steps on
512,000 unknowns), so that a test can compare them with the printed values.

- Table 12 (section "Problem 4", the degradation table): Problem 4 on 40x40x40, D = 1e4,
  convection 100, 200, 500 and 1000; Bi-CGSTAB and GMRES(10), each without and with GS(2),
  without and with ILU(0); rel-res goals 1e-4, 1e-7, 1e-10.
- The ILUT rows of the Problem 4 iteration table (80x80x80, D = 1e4 and 1e6): Bi-CGSTAB and
  GMRES(10) with ILU(0), without and with GS(2).

Every run starts from x0 = 0 with at most 10,000 iterations; runs without GS stop on the
GS(2)-scaled residual (stop weights 1/||a_i||_2). Each goal is a run of its own; once a run
fails a goal, the stricter goals are recorded as failed at the same level without running.
Calls only the oracle. Usage: python tests/golden/make_paper_tables_oracle.py [processes]
"""
import json
import os
import sys
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

TOLS = (1e-4, 1e-7, 1e-10)


def _system(kind, N, D, conv):
    from paper_0812_2769_amd import problems
    return problems.problem4(N, D=D, conv=conv)


def run_one(job):
    import numpy as np
    import oracle
    key, (N, D, conv), method, gs, ilu = job
    P = _system("p4", N, D, conv)
    vo, bo, nrm, _ = oracle.gs_scale(P, P.b, 2)
    if gs:
        A = P.copy()
        A.val, A.b = vo, bo
        b, W = bo, None
    else:
        A, b, W = P, P.b, 1.0 / nrm
    lu = oracle.ilu0(A) if ilu else None
    out = []
    failed = None
    for tol in TOLS:
        if failed is not None:
            out.append(failed)
            continue
        if method == "bicgstab":
            _, info = oracle.bicgstab(A, b, tol=tol, weights=W, ilu=lu)
        else:
            _, info = oracle.gmres(A, b, m=10, tol=tol, weights=W, ilu=lu)
        if info.status == oracle.CONVERGED:
            out.append({"iters": info.iters})
        else:
            failed = {"iters": None, "status": info.status_name,
                      "relres_true": float(info.relres_true)}
            out.append(failed)
    print(f"{key}: {out}", flush=True)
    return key, out


def jobs():
    out = []
    for conv in (100.0, 200.0, 500.0, 1000.0):
        for method in ("bicgstab", "gmres10"):
            for ilu in (False, True):
                for gs in (False, True):
                    name = f"table12/c{int(conv)}/{method}{'_ilut' if ilu else ''}{'_gs' if gs else ''}"
                    out.append((name, (40, 1e4, conv), method, gs, ilu))
    for D in (1e4, 1e6):
        for method in ("bicgstab", "gmres10"):
            for gs in (False, True):
                name = f"problem4_80/D{D:g}/{method}_ilut{'_gs' if gs else ''}"
                out.append((name, (80, D, 100.0), method, gs, True))
    return out


def main():
    procs = int(sys.argv[1]) if len(sys.argv) > 1 else 4
    with Pool(procs) as pool:
        results = dict(pool.map(run_one, jobs(), chunksize=1))
    path = os.path.join(HERE, "paper_tables_oracle.json")
    with open(path, "w") as f:
        json.dump({"note": "written by tests/golden/make_paper_tables_oracle.py (oracle only)",
                   "tols": list(TOLS), "runs": results}, f, indent=1, sort_keys=True)
    print(path)


if __name__ == "__main__":
    main()
