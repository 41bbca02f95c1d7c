"""Bases of 2 GiB and more (maximum sizes) through the C ABI.

Basis columns are read through one 32-bit buffer descriptor while the basis is under 2^31
bytes, and with plain 64-bit addresses from there on. The two forms run the same arithmetic,
so a run whose basis crosses 2^31 bytes must give bit for bit what the other form gives for
the steps they share:
- gsk_arnoldi with m = 64 (basis of 65 columns, 64-bit addressing) against m = 60 (61 columns,
  under 2^31 bytes): equal first 61 columns and Hessenberg entries; the 64-step basis is also
  checked for orthonormality and the Arnoldi relation A V_m = V_{m+1} H (properties that hold
  at any size, since the oracle is too slow at 4 M unknowns);
- GMRES(64) and GMRES(60) stopped at 60 Arnoldi steps (one cycle either way), FP64 at 162^3
  and mixed precision (FP32 basis) at 203^3: equal x and equal info.
"""
import numpy as np
import pytest

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


def scaled_stencil(G, N):
    P = problems.slabs_3d(N)
    A = G.CsrMatrix.from_problem(P)
    As, bs, _, _ = G.gs_scale(A, dev(P.b), 2)
    return G.stencil_from_csr(As, N, N, N), bs


def test_arnoldi_basis_beyond_2gib(G):
    import torch
    N = 162
    M, b = scaled_stencil(G, N)
    n = M.n
    assert 61 * 8 * n < 2 ** 31 <= 65 * 8 * n
    V60, H60, k60 = G.arnoldi(M, b, 60)
    V64, H64, k64 = G.arnoldi(M, b, 64)
    assert (k60, k64) == (60, 64)
    assert torch.equal(V60, V64[:, :61]) and torch.equal(H60, H64[:61, :60])
    del V60
    Vs = V64.t()                      # (65, n), contiguous rows: the stored columns
    gram = torch.mm(Vs, Vs.t())
    orth = (gram - torch.eye(65, dtype=gram.dtype, device=gram.device)).abs().max().item()
    assert orth <= 1e-11, orth
    worst = 0.0
    for j in range(64):
        y = G.spmv(M, Vs[j].contiguous())
        r = y - torch.mv(Vs[:j + 2].t(), H64[:j + 2, j].contiguous())
        worst = max(worst, (r.norm() / y.norm()).item())
    assert worst <= 1e-11, worst


@pytest.mark.parametrize("precision,N", [("fp64", 162), ("mixed", 203)])
def test_gmres_basis_beyond_2gib(G, precision, N):
    import torch
    M, b = scaled_stencil(G, N)
    width = 8 if precision == "fp64" else 4
    assert 61 * width * M.n < 2 ** 31 <= 65 * width * M.n
    f = G.gmres if precision == "fp64" else G.gmres_mixed
    x60, i60 = f(M, b, m=60, tol=1e-12, maxit=60)
    x64, i64 = f(M, b, m=64, tol=1e-12, maxit=60)
    assert i60 == i64 and i60.iters == 60, (i60, i64)
    assert torch.equal(x60, x64)
    assert i60.relres_true < 1.0
