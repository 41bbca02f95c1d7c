"""Structured 5/7-point stencil operator (gsk_matrix kind GSK_MATRIX_STENCIL) through the C ABI.

The stencil product sums the same products in the same order as CSR storage order of a
finite-difference matrix (columns ascending: -z, -y, -x, centre, +x, +y, +z), so it must equal
the oracle's CSR product bit for bit, and every solver must return bit-identical results and
the same iteration counts on either representation of the same matrix.
"""
import numpy as np
import pytest

import oracle
from paper_0812_2769_amd import problems

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0812_2769_amd import gsk
    return gsk


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def grid_of(P):
    d = list(P.dims) + [1] * (3 - len(P.dims))
    return d[0], d[1], d[2]


def oracle_planes(P):
    """Coefficient planes written straight from the definition of the layout (CPU, numpy)."""
    nx, ny, nz = grid_of(P)
    offs = ([-nx * ny] if nz > 1 else []) + [-nx, -1, 0, 1, nx] + ([nx * ny] if nz > 1 else [])
    planes = np.zeros((len(offs), P.n))
    for i in range(P.n):
        for k in range(P.row_ptr[i], P.row_ptr[i + 1]):
            planes[offs.index(int(P.col_idx[k]) - i), i] = P.val[k]
    return planes.ravel()


CASES = {
    "slabs_3d_14": lambda: problems.slabs_3d(14),
    "c1_2d_33": lambda: problems.square_jump_2d(33),
    "ragged_3d": lambda: problems.laplacian((13, 11, 7), conv=(40.0, -25.0, 10.0)),
    "ragged_2d": lambda: problems.laplacian((37, 29), conv=(30.0, 5.0)),
    "thin_2x2x3": lambda: problems.laplacian((2, 2, 3)),
    "p4_12": lambda: problems.problem4(12),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_pack_and_spmv_bitwise(G, case):
    P = CASES[case]()
    nx, ny, nz = grid_of(P)
    A = G.CsrMatrix.from_problem(P)
    S = G.stencil_from_csr(A, nx, ny, nz)
    assert np.array_equal(S.coef.cpu().numpy(), oracle_planes(P))
    rng = np.random.default_rng(5)
    x = rng.standard_normal(P.n)
    y = G.spmv(S, dev(x)).cpu().numpy()
    assert np.array_equal(y, oracle.spmv(P, x))
    assert np.array_equal(y, G.spmv(A, dev(x)).cpu().numpy())


def _scaled_pair(G, P, p):
    nx, ny, nz = grid_of(P)
    A = G.CsrMatrix.from_problem(P)
    As, bs, _, w = G.gs_scale(A, dev(P.b), p, want_weights=(p != 2))
    return As, G.stencil_from_csr(As, nx, ny, nz), bs, w


@pytest.mark.parametrize("case,p", [("slabs_3d_14", 2), ("slabs_3d_14", 1), ("ragged_3d", 2),
                                    ("c1_2d_33", 2), ("ragged_2d", 1)])
def test_solvers_identical_on_stencil(G, case, p):
    P = CASES[case]()
    As, Ss, bs, w = _scaled_pair(G, P, p)
    for run in (lambda M: G.gmres(M, bs, m=20, tol=1e-10, maxit=3000, stop_weights=w),
                lambda M: G.bicgstab(M, bs, tol=1e-10, maxit=3000, stop_weights=w)):
        xc, ic = run(As)
        xs, is_ = run(Ss)
        assert ic.status == is_.status   # GMRES(20) on the 2D jump problem hits maxit on both
        assert (ic.iters, ic.restarts, ic.half_step) == (is_.iters, is_.restarts, is_.half_step)
        assert np.array_equal(xc.cpu().numpy(), xs.cpu().numpy())
        assert ic.relres_true == is_.relres_true


def test_arnoldi_identical_on_stencil(G):
    P = CASES["ragged_3d"]()
    As, Ss, bs, _ = _scaled_pair(G, P, 2)
    Vc, Hc, kc = G.arnoldi(As, bs, 12)
    Vs, Hs, ks = G.arnoldi(Ss, bs, 12)
    assert kc == ks == 12
    assert np.array_equal(Vc.cpu().numpy(), Vs.cpu().numpy())
    assert np.array_equal(Hc.cpu().numpy(), Hs.cpu().numpy())


def test_stencil_solution_matches_oracle(G):
    """The stencil path against the oracle directly (same bar as the CSR solver parity)."""
    P = problems.slabs_3d(16)
    S_ref = P.copy()
    S_ref.val, S_ref.b, _, _ = oracle.gs_scale(P, P.b, 2)
    xo, io = oracle.gmres(S_ref, S_ref.b, m=30, tol=1e-10, maxit=3000)
    _, Ss, bs, _ = _scaled_pair(G, P, 2)
    xg, ig = G.gmres(Ss, bs, m=30, tol=1e-10, maxit=3000)
    assert ig.status == io.status == G.CONVERGED
    assert abs(ig.iters - io.iters) <= max(1, 0.05 * io.iters)
    xg = xg.cpu().numpy()
    assert np.max(np.abs(xg - xo)) <= 1e-8 * np.max(np.abs(xo))


def test_pack_rejects_non_stencil(G):
    P = problems.random_sparse(1000, 5, 3)
    A = G.CsrMatrix.from_problem(P)
    with pytest.raises(G.GskError) as e:
        G.stencil_from_csr(A, 10, 10, 10)
    assert e.value.code == G.ERR_INVALID_ARG
    # wrapped x neighbour: column i+1 at the end of a grid line is not a stencil position
    L = problems.laplacian((8, 8))
    rp, ci, val = L.row_ptr.copy(), L.col_idx.copy(), L.val.copy()
    i = 7                                   # last point of the first grid line
    k = rp[i + 1] - 1                       # its largest column (+y)
    ci[k] = i + 1
    bad = problems.Problem("wrap", L.dims, rp, ci, val, L.b.copy())
    with pytest.raises(G.GskError):
        G.stencil_from_csr(G.CsrMatrix.from_problem(bad), 8, 8, 1)
    with pytest.raises(G.GskError):         # grid does not match n
        G.stencil_from_csr(G.CsrMatrix.from_problem(L), 8, 7, 1)
