"""Pins of the GS(p) oracle against what the paper and the mathematics fix.

GS(p) (section 1; section 2, eq. (2)): row i of A and b_i are divided by ||a_i||_p, so that
every row of the scaled matrix has unit Lp-norm, and the scaled system has the same solution.
"""
import os

import numpy as np
import pytest

import oracle
from paper_0812_2769_amd import problems

HERE = os.path.dirname(os.path.abspath(__file__))


def _rows(P, val):
    return [val[P.row_ptr[i]:P.row_ptr[i + 1]] for i in range(P.n)]


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("seed", [0, 1])
def test_scaled_rows_have_unit_norm(p, seed):
    P = problems.random_sparse(300, 5, seed)
    vo, bo, nrm, w = oracle.gs_scale(P, P.b, p)
    for i, row in enumerate(_rows(P, vo)):
        assert np.linalg.norm(row, ord=p) == pytest.approx(1.0, rel=8e-16 * len(row) + 1e-16)
    # norms agree with numpy's vector p-norm of the unscaled rows
    ref = np.array([np.linalg.norm(r, ord=p) for r in _rows(P, P.val)])
    np.testing.assert_allclose(nrm, ref, rtol=4e-16 * 8, atol=0)
    # b scaled by the same factors
    np.testing.assert_allclose(bo * nrm, P.b, rtol=2e-16, atol=0)


def test_closed_forms_2d_3d():
    # 2D Laplacian (a = 1, no convection): interior row [4,-1,-1,-1,-1]; corner row [4,-1,-1].
    L = problems.laplacian((5, 5))
    vo, _, _, _ = oracle.gs_scale(L, L.b, 2)
    rows = _rows(L, vo)
    interior = rows[12]          # node (2,2)
    assert len(interior) == 5
    np.testing.assert_allclose(sorted(interior), sorted([4 / np.sqrt(20)] + [-1 / np.sqrt(20)] * 4),
                               rtol=1e-15)
    assert max(interior) == pytest.approx(0.894427191, abs=1e-9)
    assert min(interior) == pytest.approx(-0.223606798, abs=1e-9)
    corner = rows[0]
    np.testing.assert_allclose(sorted(corner), sorted([4 / np.sqrt(18), -1 / np.sqrt(18), -1 / np.sqrt(18)]),
                               rtol=1e-15)
    assert max(corner) == pytest.approx(0.942809042, abs=1e-9)
    # p = 1: divide by the absolute row sum (AZTEC's "row-sum scaling")
    v1, _, _, _ = oracle.gs_scale(L, L.b, 1)
    r1 = _rows(L, v1)
    np.testing.assert_allclose(sorted(r1[12]), sorted([0.5] + [-0.125] * 4), rtol=1e-15)
    np.testing.assert_allclose(sorted(r1[0]), sorted([4 / 6, -1 / 6, -1 / 6]), rtol=1e-15)
    # 3D interior row [6, -1 x 6] / sqrt(42)
    L3 = problems.laplacian((4, 4, 4))
    v3, _, _, _ = oracle.gs_scale(L3, L3.b, 2)
    r3 = _rows(L3, v3)[1 + 4 + 16]   # node (1,1,1)
    assert len(r3) == 7
    assert max(r3) == pytest.approx(0.925820100, abs=1e-9)
    assert min(r3) == pytest.approx(-0.154303350, abs=1e-9)
    v31, _, _, _ = oracle.gs_scale(L3, L3.b, 1)
    assert max(_rows(L3, v31)[21]) == pytest.approx(0.5, abs=1e-15)


def test_convection_row_closed_form():
    # 2D, a = 1, constant convection (c1, c2) = (10, 10), N = 9 (h = 0.1): interior row
    # [-1 - c h/2 (-y), -1 - c h/2 (-x), 4, -1 + c h/2 (+x), -1 + c h/2 (+y)]
    L = problems.laplacian((9, 9), conv=(10.0, 10.0))
    row = _rows(L, L.val)[4 + 9 * 4]
    np.testing.assert_allclose(row, [-1.5, -1.5, 4.0, -0.5, -0.5], rtol=1e-15)
    vo, _, nrm, _ = oracle.gs_scale(L, L.b, 2)
    assert nrm[4 + 9 * 4] == pytest.approx(np.sqrt(2 * 1.5 ** 2 + 16 + 2 * 0.25), rel=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_positive_row_scaling_invariance(p):
    P = problems.random_sparse(200, 6, 5)
    rng = np.random.default_rng(11)
    s = 10.0 ** rng.uniform(-3, 3, size=P.n)
    Q = P.copy()
    Q.val = P.val * np.repeat(s, np.diff(P.row_ptr))
    Q.b = P.b * s
    v1, b1, _, _ = oracle.gs_scale(P, P.b, p)
    v2, b2, _, _ = oracle.gs_scale(Q, Q.b, p)
    np.testing.assert_allclose(v2, v1, rtol=1e-14, atol=0)
    np.testing.assert_allclose(b2, b1, rtol=1e-14, atol=0)
    # sign: scaling by -1 flips the scaled row
    Q.val = -P.val
    v3, _, _, _ = oracle.gs_scale(Q, -P.b, p)
    np.testing.assert_array_equal(v3, -v1)


@pytest.mark.parametrize("p", [1, 2])
def test_idempotent(p):
    P = problems.square_jump_2d(16)
    v1, b1, _, _ = oracle.gs_scale(P, P.b, p)
    Q = P.copy()
    Q.val, Q.b = v1, b1
    v2, b2, n2, _ = oracle.gs_scale(Q, b1, p)
    np.testing.assert_allclose(n2, 1.0, rtol=1e-15)
    np.testing.assert_allclose(v2, v1, rtol=4e-16, atol=0)


@pytest.mark.parametrize("maker", [lambda: problems.square_jump_2d(10), lambda: problems.problem4(5, 1e4),
                                   lambda: problems.slabs_3d(5)])
def test_scaling_keeps_the_solution(maker):
    # D A x = D b has the solution of A x = b (section 2, eq. (2)); dense LU as the referee.
    P = maker()
    A = P.dense()
    x = np.linalg.solve(A, P.b)
    for p in (1, 2):
        vo, bo, _, _ = oracle.gs_scale(P, P.b, p)
        Q = P.copy()
        Q.val = vo
        xs = np.linalg.solve(Q.dense(), bo)
        np.testing.assert_allclose(xs, x, rtol=1e-10, atol=1e-12 * np.abs(x).max())


def test_weights_convert_to_the_gs2_metric():
    P = problems.slabs_3d(6)
    _, _, n1, w1 = oracle.gs_scale(P, P.b, 1)
    _, _, n2, w2 = oracle.gs_scale(P, P.b, 2)
    np.testing.assert_array_equal(w2, np.ones(P.n))
    l2 = np.array([np.linalg.norm(r) for r in _rows(P, P.val)])
    np.testing.assert_allclose(w1, n1 / l2, rtol=1e-15)
    # Cauchy-Schwarz: ||a||_2 <= ||a||_1 <= sqrt(k) ||a||_2
    k = np.diff(P.row_ptr)
    assert np.all(w1 >= 1 - 1e-15) and np.all(w1 <= np.sqrt(k) + 1e-15)


def test_errors():
    P = problems.random_sparse(20, 3, 2)
    Z = P.copy()
    Z.val[Z.row_ptr[7]:Z.row_ptr[8]] = 0.0
    with pytest.raises(oracle.OracleError) as e:
        oracle.gs_scale(Z, Z.b, 2)
    assert e.value.code == oracle.ERR_ZERO_ROW
    N = P.copy()
    N.val[3] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        oracle.gs_scale(N, N.b, 2)
    assert e.value.code == oracle.ERR_NONFINITE
    B = P.copy()
    B.b[5] = np.inf
    with pytest.raises(oracle.OracleError) as e:
        oracle.gs_scale(B, B.b, 1)
    assert e.value.code == oracle.ERR_NONFINITE
    with pytest.raises(oracle.OracleError) as e:
        oracle.gs_scale(P, P.b, 0)
    assert e.value.code == oracle.ERR_ARG


def _read_golden(name):
    rows = {}
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            rows[parts[0]] = parts[1:]
    return rows


@pytest.mark.slow
def test_table3_eigenvalues_reproduced():
    """Generator + GS(2) oracle reproduce Table 3 (Problem 1, 40x40): 3 printed digits."""
    gold = _read_golden("table3_problem1_eigen.txt")
    P = problems.problem1(40)
    C = problems.problem1(40, continuous=1000.0)
    vo, _, _, _ = oracle.gs_scale(P, P.b, 2)
    S = P.copy()
    S.val = vo
    for key, M in (("original", P.dense()), ("gs2", S.dense()), ("continuous", C.dense())):
        ev = np.abs(np.linalg.eigvals(M))
        lo, hi = ev.min(), ev.max()
        counts, _ = np.histogram(ev, bins=100)
        g = gold[key]
        assert lo == pytest.approx(float(g[0]), rel=0.01), key
        assert hi == pytest.approx(float(g[1]), rel=0.01), key
        assert hi / lo == pytest.approx(float(g[2]), rel=0.01), key
        assert counts[0] == int(g[3]), key
