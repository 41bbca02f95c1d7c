"""The paper's convergence tables reproduced by the oracle (CPU).

- Table 2 (Problem 1 with a = b = 1000 everywhere, 128x128), computed here.
- The ILUT rows of Tables 1 and 2, computed here with the oracle's ILU(0) (the paper's ILUT
  parameters are not printed; ILU(0) is the oracle's cross-check preconditioner).
- Table 12 (Problem 4, 40x40x40, D = 1e4, convection 100..1000) and the ILUT rows of the
  Problem 4 table (80x80x80): too slow to recompute in this suite, so they are read from
  tests/golden/paper_tables_oracle.json, which tests/golden/make_paper_tables_oracle.py writes
  by calling only the oracle.

Every run starts from x0 = 0, stops on the GS(2)-scaled residual (runs without GS through stop
weights 1/||a_i||_2), GMRES restarts every 10 steps, at most 10,000 iterations. Printed values
are in tests/golden/*.txt with their citations.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_0812_2769_amd import problems

HERE = os.path.dirname(os.path.abspath(__file__))
TOLS = (1e-4, 1e-7, 1e-10)


def _printed(name):
    rows = {}
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                parts = line.split()
                rows[parts[0]] = parts[1:]
    return rows


def _operators(P):
    """(unscaled system, b, stop weights) and (GS(2)-scaled system, b, None)."""
    vo, bo, nrm, _ = oracle.gs_scale(P, P.b, 2)
    S = P.copy()
    S.val, S.b = vo, bo
    return {"": (P, P.b, 1.0 / nrm), "_gs": (S, bo, None)}


def _solve(method, A, b, W, tol, lu):
    if method == "bicgstab":
        return oracle.bicgstab(A, b, tol=tol, weights=W, ilu=lu)[1]
    return oracle.gmres(A, b, m=10, tol=tol, weights=W, ilu=lu)[1]


def _goals(method, A, b, W, lu):
    """One run per goal; after a failed goal the stricter ones fail at the same level."""
    out, failed = [], None
    for tol in TOLS:
        if failed is None:
            info = _solve(method, A, b, W, tol, lu)
            if info.status != oracle.CONVERGED:
                failed = info
            out.append(info)
        else:
            out.append(failed)
    return out


def test_table2_problem1_continuous():
    """All runs of Table 2 converge at every goal. Without a preconditioner the counts lie
    within 10% of the printed ones (GMRES(10) equals them or nearly so), except Bi-CGSTAB
    with GS at 1e-10, whose count moves between 259 and 309 under 1-ulp perturbations of the
    data: there the median of 15 perturbed runs must be within 10% of the printed 261. With
    ILU(0) in place of the paper's ILUT, GMRES(10) must be within 5% (it equals the printed
    140 / 359 / 579) and Bi-CGSTAB within 15%."""
    gold = _printed("table2_problem1_continuous_iterations.txt")
    P = problems.problem1(128, continuous=1000.0)
    ops = _operators(P)
    for key, (A, b, W) in ops.items():
        lu = oracle.ilu0(A)
        for method in ("bicgstab", "gmres10"):
            for pre, L in (("", None), ("_ilut", lu)):
                name = method + pre + key
                infos = _goals(method, A, b, W, L)
                for t, info in enumerate(infos):
                    assert info.status == oracle.CONVERGED, (name, TOLS[t], info)
                    printed = int(gold[name][t])
                    if name == "bicgstab_gs" and t == 2:
                        continue
                    rel = 0.15 if name.startswith("bicgstab_ilut") else \
                        0.05 if pre else 0.10
                    assert info.iters == pytest.approx(printed, rel=rel), (name, TOLS[t], info)
    S, bs, _ = ops["_gs"]
    its = []
    for k in range(15):
        rng = np.random.default_rng(3000 + k)
        T = S.copy()
        T.val = S.val * (1 + 2.2e-16 * rng.choice([-1, 0, 1], size=S.nnz))
        T.b = bs * (1 + 2.2e-16 * rng.choice([-1, 0, 1], size=S.n))
        info = oracle.bicgstab(T, T.b, tol=1e-10)[1]
        assert info.status == oracle.CONVERGED
        its.append(info.iters)
    assert np.median(its) == pytest.approx(int(gold["bicgstab_gs"][2]), rel=0.10), sorted(its)


def test_table1_ilut_rows():
    """Table 1's ILUT rows with ILU(0): Bi-CGSTAB within 5% of the printed counts, without and
    with GS; GMRES(10) stagnates without GS at the printed level (3.9e-3) and with GS reaches
    1e-4 in the printed 39 steps, then stagnates at the printed 1.1e-5 (levels within a factor
    1.5)."""
    gold = _printed("ilut_rows_iterations.txt")
    ops = _operators(problems.problem1(128))
    for key, (A, b, W) in ops.items():
        lu = oracle.ilu0(A)
        for t, info in enumerate(_goals("bicgstab", A, b, W, lu)):
            assert info.status == oracle.CONVERGED
            assert info.iters == pytest.approx(int(gold["p1_bicgstab_ilut" + key][t]), rel=0.05)
        row = gold["p1_gmres10_ilut" + key]
        for t, info in enumerate(_goals("gmres10", A, b, W, lu)[:2]):
            if row[t].startswith("->"):
                level = float(row[t][2:])
                assert info.status != oracle.CONVERGED
                assert level / 1.5 < info.relres_true < level * 1.5, (key, info)
            else:
                assert info.status == oracle.CONVERGED
                assert info.iters == pytest.approx(int(row[t]), rel=0.05), (key, info)


def _oracle_runs():
    with open(os.path.join(HERE, "golden", "paper_tables_oracle.json")) as f:
        return json.load(f)["runs"]


def _best(runs):
    best = "none"
    for tol, r in zip(("1e-4", "1e-7", "1e-10"), runs):
        if r["iters"] is not None:
            best = tol
    return best


def test_table12_goals_from_the_oracle():
    """Table 12: the strictest goal each of the eight methods reaches at convection 100, 200,
    500 and 1000.
    - The four rows without ILU equal the printed ones in every cell but one. GMRES(10) with GS
      at convection 500 reaches 1e-4 in the oracle (163 steps) and then stagnates at 6.0e-5,
      just below the goal, where the paper reports no goal at all; the level is required to
      lie within a factor 2 of 1e-4 (a borderline case of restarted GMRES's stagnation, which
      the discretisation's rounding shifts).
    - The four ILU rows, with ILU(0) in place of the paper's ILUT, equal the printed ones in
      14 of 16 cells. At convection 200 Bi-CGSTAB with ILU(0) reaches 1e-10 (97 iterations,
      with and without GS) where the paper's ILUT stops at 1e-4; the ILUT drop tolerance and
      fill are not printed, so the two factorisations differ."""
    gold = _printed("table12_problem4_40cube_goals.txt")
    runs = _oracle_runs()
    for c_i, conv in enumerate((100, 200, 500, 1000)):
        for method, row in gold.items():
            r = runs[f"table12/c{conv}/{method}"]
            got = _best(r)
            if method == "gmres10_gs" and conv == 500:
                assert got == "1e-4" and 5e-5 < r[1]["relres_true"] < 2e-4, r
                continue
            if method.startswith("bicgstab_ilut") and conv == 200:
                assert row[c_i] == "1e-4" and got == "1e-10", r
                continue
            assert got == row[c_i], (conv, method, got, row[c_i])


def test_problem4_80_ilut_rows_from_the_oracle():
    """The ILUT rows of the Problem 4 table (80x80x80) with ILU(0) in place of the paper's
    ILUT, whose drop tolerance and fill are not printed.
    - Bi-CGSTAB+ILU converges to every goal at both D, and GS shortens the run to 1e-10, as
      printed. With GS the loose goals take the printed counts (13 steps to 1e-4 at both D, 19
      to 1e-7 at D = 1e6, within 5%), and so does 1e-10 at D = 1e4 (81 against 84). The other
      counts differ from the printed ones by up to a factor of two (37 against 77 steps to
      1e-4 at D = 1e4 without GS; 114 against 86 to 1e-10 at D = 1e6 with GS).
    - GMRES(10)+ILU: the converge / no-converge pattern equals the printed one in 11 of 12
      cells, and converged counts with GS are within 5% (29 / 47 against 28 / 46). The cell
      that differs is D = 1e4 without GS at 1e-4: ILU(0) gets there after 3,850 of the 10,000
      steps, where the paper's ILUT did not; both stall before 1e-7."""
    gold = _printed("ilut_rows_iterations.txt")
    runs = _oracle_runs()
    for D in ("1e4", "1e6"):
        plain = runs[f"problem4_80/D{float(D):g}/bicgstab_ilut"]
        gs = runs[f"problem4_80/D{float(D):g}/bicgstab_ilut_gs"]
        assert all(r["iters"] is not None for r in plain + gs)
        assert gs[2]["iters"] < plain[2]["iters"]
        row = gold[f"p4_D{D}_bicgstab_ilut_gs"]
        assert gs[0]["iters"] == pytest.approx(int(row[0]), rel=0.05), gs
        if D == "1e6":
            assert gs[1]["iters"] == pytest.approx(int(row[1]), rel=0.05), gs
        else:
            assert gs[2]["iters"] == pytest.approx(int(row[2]), rel=0.05), gs
        for suffix in ("", "_gs"):
            r = runs[f"problem4_80/D{float(D):g}/gmres10_ilut{suffix}"]
            prow = gold[f"p4_D{D}_gmres10_ilut{suffix}"]
            for t in range(3):
                if (D, suffix, t) == ("1e4", "", 0):
                    assert prow[t] == "nc" and r[t]["iters"] > 3000, r
                    continue
                assert (r[t]["iters"] is None) == (prow[t] == "nc"), (D, suffix, t, r)
                if r[t]["iters"] is not None:
                    assert r[t]["iters"] == pytest.approx(int(prow[t]), rel=0.05), (D, suffix, r)
