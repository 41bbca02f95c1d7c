"""Write tests/golden/slabs80_oracle.json: the FP64 oracle's results on the 80^3 benchmark system.

Calls only the oracle (and the seeded generator). Re-run after any change to the oracle's
arithmetic or to the generator: `python tests/golden/make_slabs80_golden.py`. Takes ~2 minutes.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_0812_2769_amd import problems  # noqa: E402

SAMPLE_SEED = 7
N_SAMPLE = 512


def main():
    P = problems.slabs_3d()
    idx = np.sort(np.random.default_rng(SAMPLE_SEED).choice(P.n, size=N_SAMPLE, replace=False))
    out = {"workload": "80^3, 8 log-uniform slabs (seed 1002), convection (20,-10,5)",
           "n": P.n, "nnz": P.nnz, "sample_seed": SAMPLE_SEED, "sample_idx": idx.tolist(),
           "runs": {}}
    for p in (2, 1):
        vo, bo, nrm, w = oracle.gs_scale(P, P.b, p)
        S = P.copy()
        S.val, S.b = vo, bo
        W = None if p == 2 else w
        for method in ("bicgstab", "gmres30"):
            t = time.time()
            if method == "bicgstab":
                x, info = oracle.bicgstab(S, bo, tol=1e-10, weights=W)
            else:
                x, info = oracle.gmres(S, bo, m=30, tol=1e-10, weights=W)
            key = f"gs{p}_{method}"
            out["runs"][key] = {
                "iters": info.iters, "restarts": info.restarts, "status": info.status,
                "relres_true": info.relres_true, "x_sample": x[idx].tolist(),
                "x_norm": float(np.linalg.norm(x)),
                "err_vs_u_star": float(np.linalg.norm(x - P.u_star) / np.linalg.norm(P.u_star)),
                "oracle_seconds": time.time() - t}
            print(key, info, f"{time.time() - t:.1f}s", flush=True)
    with open(os.path.join(HERE, "slabs80_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
