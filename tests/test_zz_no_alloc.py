"""gsk_bicgstab_noalloc (Bi-CGSTAB in the library's fixed scratch array, no allocation)
against gsk_bicgstab (caller's workspace) through the C ABI: the same launches, so results must
be equal bit for bit (x, iteration and restart counts, status, both residuals). Two calls in
a row on one GPU share the scratch array; the second, smaller system must not see the first
one's leftovers."""
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


def scaled(G, P, p=2, stencil=True):
    A = G.CsrMatrix.from_problem(P)
    As, bs, _, w = G.gs_scale(A, dev(P.b), p, want_weights=(p != 2))
    d = list(P.dims) + [1] * (3 - len(P.dims))
    M = G.stencil_from_csr(As, *d) if stencil else As
    return M, bs, (w if p != 2 else None)


def check_equal(G, M, b, w, tol):
    import torch
    x_ref, i_ref = G.bicgstab(M, b, tol=tol, stop_weights=w)
    x = torch.zeros_like(b)
    info = G.bicgstab_noalloc(M, b, x, tol=tol, stop_weights=w)
    torch.cuda.synchronize()
    assert info == i_ref, (info, i_ref)
    assert info.status == G.CONVERGED
    assert torch.equal(x, x_ref)


def test_noalloc_two_calls_equal_workspace_path(G):
    # first call: 80^3 slabs (512,000 rows, the largest benchmark system that fits the
    # scratch array); second call: a smaller batch-recipe system
    big = scaled(G, problems.slabs_3d(80))
    check_equal(G, *big, tol=1e-10)
    small = scaled(G, problems.batch_system(problems.batch_specs(1, seed=21, n_min=17,
                                                                 n_max=17)[0]))
    check_equal(G, *small, tol=1e-10)


def test_noalloc_csr_weights_and_ragged(G):
    # GS(1) with stop weights, then a CSR matrix, then a tiny ragged system, each after a
    # larger one
    check_equal(G, *scaled(G, problems.slabs_3d(30), p=1), tol=1e-10)
    check_equal(G, *scaled(G, problems.laplacian((21, 13, 5), conv=(9.0, -4.0, 2.0)),
                           stencil=False), tol=1e-10)
    check_equal(G, *scaled(G, problems.laplacian((3, 2))), tol=1e-12)


def test_noalloc_rejects_systems_beyond_the_scratch_size(G):
    import torch
    N = 100                          # 10^6 rows: about 57 MB of Bi-CGSTAB workspace
    n = N ** 3
    need = G.workspace_bytes(G.METHOD_BICGSTAB, n)
    assert need > G.bicgstab_noalloc_max_bytes()
    M = G.StencilMatrix(N, N, N, torch.zeros(7 * n, dtype=torch.float64, device="cuda"))
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(G.GskError) as e:
        G.bicgstab_noalloc(M, b, x, tol=1e-8)
    assert e.value.code == G.ERR_WORKSPACE
    assert not x.any()
