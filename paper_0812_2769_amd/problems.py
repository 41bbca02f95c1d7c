"""Seeded synthetic convection-diffusion systems: the inputs of every test and benchmark.

This module builds matrices and right-hand sides only. It holds none of the arithmetic of
geometric scaling or of the Krylov solvers, and it imports neither the HIP library nor the
oracle, so both sides can be fed from here.

Discretisation (section "Setup of the numerical experiments", the eqnarray for the flux of
(a u_x)_x): second-order terms in flux form with the coefficient evaluated at the face
midpoint between two nodes; first-order terms by central differences of the flux c*u with c
taken at the neighbouring node; Dirichlet neighbours are dropped from the matrix and their
boundary value is moved into the right-hand side. Every row is multiplied by h^2 (the form
whose eigenvalues the paper tabulates for Problem 1, Table 3). Interior nodes only; node k of
an axis with N nodes sits at (k+1)h with h = 1/(N+1), and the face between nodes f-1 and f
sits at (f+1/2)h.

Positions are carried as integers q over a denominator den = 2(N+1): node k has q = 2(k+1),
face f has q = 2f+1. Region tests such as 1/4 < x < 3/4 are then exact integer comparisons,
and cells of a partition are half-open [lo, hi) with no floating-point tie at a boundary.

Row order is x fastest, then y, then z; within a row the columns are ascending
(-z, -y, -x, diagonal, +x, +y, +z).
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional, Sequence

import numpy as np

__all__ = [
    "Problem",
    "assemble",
    "problem1",
    "problem4",
    "square_jump_2d",
    "slabs_3d",
    "checkerboard_3d",
    "laplacian",
    "random_sparse",
]


@dataclasses.dataclass
class Problem:
    """A sparse system A x = b in CSR form (FP64 values, int32 indices)."""

    name: str
    dims: tuple            # interior nodes per axis, x first: (Nx, Ny) or (Nx, Ny, Nz)
    row_ptr: np.ndarray    # int32 [n+1]
    col_idx: np.ndarray    # int32 [nnz]
    val: np.ndarray        # float64 [nnz]
    b: np.ndarray          # float64 [n]
    u_star: Optional[np.ndarray] = None   # exact solution of the discrete system, if manufactured

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    def dense(self) -> np.ndarray:
        """Dense copy of A (small systems only)."""
        n = self.n
        out = np.zeros((n, n))
        rows = np.repeat(np.arange(n), np.diff(self.row_ptr))
        out[rows, self.col_idx] = self.val
        return out

    def copy(self) -> "Problem":
        return dataclasses.replace(
            self, row_ptr=self.row_ptr.copy(), col_idx=self.col_idx.copy(),
            val=self.val.copy(), b=self.b.copy(),
            u_star=None if self.u_star is None else self.u_star.copy())


# Coefficient callbacks receive integer position arrays (one per axis, x first) and the
# per-axis denominators, and return float64 arrays of the same shape.
CoefFn = Callable[[Sequence[np.ndarray], Sequence[int]], np.ndarray]


def _node_q(N: int) -> np.ndarray:
    return 2 * (np.arange(N, dtype=np.int64) + 1)


def _face_q(N: int) -> np.ndarray:
    return 2 * np.arange(N + 1, dtype=np.int64) + 1


def _grids(qs):
    """Broadcastable integer position arrays in (z, y, x) memory order, returned x first."""
    d = len(qs)
    out = []
    for axis, q in enumerate(qs):
        shape = [1] * d
        shape[d - 1 - axis] = q.shape[0]
        out.append(q.reshape(shape))
    return out


def assemble(dims: Sequence[int], diff: CoefFn, conv: Sequence, u_star_fn=None,
             boundary_fn=None, rhs_fn=None, name: str = "custom") -> Problem:
    """Assemble the h^2-scaled flux-form central-difference system on the unit square/cube.

    diff(q, den) -> diffusion coefficient at the given positions (evaluated at face midpoints).
    conv[d] is either a float (constant convection along axis d) or a callable
    conv[d](q, den) evaluated at node positions.
    u_star_fn(q, den) -> exact grid solution; if given, b = A u*.
    boundary_fn(q, den) -> Dirichlet value at boundary nodes (default 0).
    rhs_fn(q, den) -> source term F at the nodes (h^2-scaled into b); default 0.
    """
    dims = tuple(int(v) for v in dims)
    d = len(dims)
    assert d in (2, 3)
    dens = [2 * (N + 1) for N in dims]
    hs = [1.0 / (N + 1) for N in dims]
    shape = tuple(reversed(dims))           # (Nz, Ny, Nx) memory order
    n = int(np.prod(dims))
    node_q = [_node_q(N) for N in dims]
    node_grid = _grids(node_q)

    def conv_at(axis, qgrid):
        c = conv[axis]
        if callable(c):
            return np.broadcast_to(np.asarray(c(qgrid, dens), dtype=np.float64), shape)
        return np.full(shape, float(c))

    # Stencil arrays: for each axis, coefficient of the -1 and +1 neighbours, plus diagonal.
    diag = np.zeros(shape)
    lower = []   # coefficient of node - e_axis
    upper = []   # coefficient of node + e_axis
    for axis in range(d):
        N = dims[axis]
        fq = _face_q(N)
        qs = list(node_q)
        qs[axis] = fq
        face = np.broadcast_to(np.asarray(diff(_grids(qs), dens), dtype=np.float64),
                               tuple(reversed([len(q) for q in qs]))).copy()
        mem_axis = d - 1 - axis
        a_minus = np.take(face, np.arange(0, N), axis=mem_axis)       # face f = k
        a_plus = np.take(face, np.arange(1, N + 1), axis=mem_axis)    # face f = k+1
        diag = diag + a_minus + a_plus
        h = hs[axis]
        # convection coefficient taken at the neighbouring node (flux form of (c u)_axis)
        qm = list(node_q)
        qm[axis] = node_q[axis] - 2          # node k-1 (q = 2k); may be the boundary node
        qp = list(node_q)
        qp[axis] = node_q[axis] + 2          # node k+1
        c_minus = conv_at(axis, _grids(qm))
        c_plus = conv_at(axis, _grids(qp))
        lower.append(-a_minus - 0.5 * h * c_minus)
        upper.append(-a_plus + 0.5 * h * c_plus)

    # Column layout per row: ascending order -z, -y, -x, diag, +x, +y, +z
    idx = np.arange(n, dtype=np.int64).reshape(shape)
    strides = [1, dims[0], dims[0] * dims[1]][:d]
    cols = []
    vals = []
    masks = []
    for axis in reversed(range(d)):
        mem_axis = d - 1 - axis
        pos = np.arange(dims[axis]).reshape([-1 if a == mem_axis else 1 for a in range(d)])
        m = np.broadcast_to(pos > 0, shape)
        cols.append(idx - strides[axis])
        vals.append(lower[axis])
        masks.append(m)
    cols.append(idx)
    vals.append(diag)
    masks.append(np.ones(shape, dtype=bool))
    for axis in range(d):
        mem_axis = d - 1 - axis
        pos = np.arange(dims[axis]).reshape([-1 if a == mem_axis else 1 for a in range(d)])
        m = np.broadcast_to(pos < dims[axis] - 1, shape)
        cols.append(idx + strides[axis])
        vals.append(upper[axis])
        masks.append(m)
    C = np.stack([c.reshape(-1) for c in cols], axis=1)
    V = np.stack([np.broadcast_to(v, shape).reshape(-1) for v in vals], axis=1)
    M = np.stack([m.reshape(-1) for m in masks], axis=1)
    counts = M.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col_idx = C[M].astype(np.int32)
    val = np.ascontiguousarray(V[M], dtype=np.float64)

    # Right-hand side: source term, Dirichlet data moved across, or manufactured b = A u*.
    b = np.zeros(n)
    u_star = None
    if rhs_fn is not None:
        hh = hs[0] * hs[0]
        b = b + hh * np.broadcast_to(np.asarray(rhs_fn(node_grid, dens), dtype=np.float64),
                                     shape).reshape(-1)
    if boundary_fn is not None:
        for axis in range(d):
            mem_axis = d - 1 - axis
            N = dims[axis]
            for side, coef in ((0, lower[axis]), (N - 1, upper[axis])):
                qs = list(node_q)
                qs[axis] = np.array([0 if side == 0 else 2 * (N + 1)], dtype=np.int64)
                g = np.asarray(boundary_fn(_grids(qs), dens), dtype=np.float64)
                sl = [slice(None)] * d
                sl[mem_axis] = slice(side, side + 1)
                contrib = np.zeros(shape)
                contrib[tuple(sl)] = -np.take(coef, [side], axis=mem_axis) * g
                b = b + contrib.reshape(-1)
    if u_star_fn is not None:
        u_star = np.ascontiguousarray(
            np.broadcast_to(np.asarray(u_star_fn(node_grid, dens), dtype=np.float64),
                            shape).reshape(-1))
        prod = np.where(M, V * u_star[np.where(M, C, 0)], 0.0)
        b = b + prod.sum(axis=1)
    if row_ptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("nnz exceeds int32 indexing")
    return Problem(name=name, dims=dims, row_ptr=row_ptr.astype(np.int32), col_idx=col_idx,
                   val=val, b=np.ascontiguousarray(b), u_star=u_star)


# ---------------------------------------------------------------------------------------
# The paper's problems
# ---------------------------------------------------------------------------------------

def problem1(N: int = 128, jump: float = 1e3, continuous: Optional[float] = None) -> Problem:
    """Problem 1 (Saad's F2DB, section "Problem 1"): -(a u_x)_x-(a u_y)_y+(d u)_x+(e u)_y.

    a = `jump` on the open square (1/4,3/4)^2 and 1 elsewhere; with `continuous` set, a is that
    constant everywhere (the a = 1000 variant of Table 2). d = 10(x+y), e = 10(x-y), u = 0 on
    the boundary, b = A e with e the all-ones vector.
    """

    def diff(q, den):
        qx, qy = q
        if continuous is not None:
            return np.full(np.broadcast_shapes(qx.shape, qy.shape), float(continuous))
        inside = (4 * qx > den[0]) & (4 * qx < 3 * den[0]) & (4 * qy > den[1]) & (4 * qy < 3 * den[1])
        return np.where(inside, jump, 1.0)

    def d_fn(q, den):
        return 10.0 * (q[0] / den[0] + q[1] / den[1])

    def e_fn(q, den):
        return 10.0 * (q[0] / den[0] - q[1] / den[1])

    return assemble((N, N), diff, (d_fn, e_fn), u_star_fn=lambda q, den: np.ones(1),
                    name=f"problem1_N{N}")


def problem4(N: int = 40, D: float = 1e4, conv: float = 100.0) -> Problem:
    """Problem 4 (section "Problem 4"): 3D, a = D on the open cube (1/3,2/3)^3, else 1;
    convection d = e = f = conv; u = 1 on the z = 0 plane, 0 on the other faces; F = 0."""

    def diff(q, den):
        inside = np.ones(np.broadcast_shapes(*[x.shape for x in q]), dtype=bool)
        for a in range(3):
            inside &= (3 * q[a] > den[a]) & (3 * q[a] < 2 * den[a])
        return np.where(inside, D, 1.0)

    def bnd(q, den):
        qz = q[2]
        return np.where(qz == 0, 1.0, 0.0) * np.ones(np.broadcast_shapes(*[x.shape for x in q]))

    return assemble((N, N, N), diff, (conv, conv, conv), boundary_fn=bnd,
                    name=f"problem4_N{N}_D{D:g}_c{conv:g}")


# ---------------------------------------------------------------------------------------
# Benchmark workloads (synthetic, seeded)
# ---------------------------------------------------------------------------------------

def square_jump_2d(N: int = 64) -> Problem:
    """2D, 64x64 interior, a = 1e3 on the open square (1/4,3/4)^2 else 1, convection (10,10),
    b = A u* with u* = x(1-x)y(1-y)e^(x+y) on the grid. Deterministic."""

    def diff(q, den):
        qx, qy = q
        inside = (4 * qx > den[0]) & (4 * qx < 3 * den[0]) & (4 * qy > den[1]) & (4 * qy < 3 * den[1])
        return np.where(inside, 1e3, 1.0)

    def u_star(q, den):
        x = q[0] / den[0]
        y = q[1] / den[1]
        return x * (1 - x) * y * (1 - y) * np.exp(x + y)

    return assemble((N, N), diff, (10.0, 10.0), u_star_fn=u_star, name=f"square_jump_2d_N{N}")


def _sine_product(q, den):
    out = 1.0
    for a in range(len(q)):
        out = out * np.sin(np.pi * (q[a] / den[a]))
    return out


def slabs_3d(N: int = 80, seed: int = 1002, slabs: int = 8) -> Problem:
    """3D, N^3 interior, a piecewise constant on `slabs` equal slabs along z (half-open cells),
    slab values 10^U(0,6) drawn in slab order from numpy's default_rng(seed); convection
    (20,-10,5); b = A u* with u* = sin(pi x) sin(pi y) sin(pi z)."""
    rng = np.random.default_rng(seed)
    slab_val = 10.0 ** rng.uniform(0.0, 6.0, size=slabs)

    def diff(q, den):
        s = (slabs * q[2]) // den[2]
        s = np.clip(s, 0, slabs - 1)
        return np.broadcast_to(slab_val[s], np.broadcast_shapes(*[x.shape for x in q]))

    p = assemble((N, N, N), diff, (20.0, -10.0, 5.0), u_star_fn=_sine_product,
                 name=f"slabs_3d_N{N}_seed{seed}")
    return p


def checkerboard_3d(N: int = 160, seed: int = 1003, blocks_per_axis: int = 16,
                    prob: float = 0.3, high: float = 1e4) -> Problem:
    """3D, N^3 interior, random checkerboard: blocks_per_axis^3 cubes (half-open cells), each
    cube a = `high` with probability `prob` else 1, drawn as default_rng(seed).random(
    (B,B,B)) < prob indexed [bz, by, bx]; convection (5,5,5); b = A u*, u* = sine product."""
    rng = np.random.default_rng(seed)
    B = blocks_per_axis
    field = np.where(rng.random((B, B, B)) < prob, high, 1.0)

    def diff(q, den):
        bx = np.clip((B * q[0]) // den[0], 0, B - 1)
        by = np.clip((B * q[1]) // den[1], 0, B - 1)
        bz = np.clip((B * q[2]) // den[2], 0, B - 1)
        return field[bz, by, bx]

    return assemble((N, N, N), diff, (5.0, 5.0, 5.0), u_star_fn=_sine_product,
                    name=f"checkerboard_3d_N{N}_seed{seed}")


def batch_specs(count: int = 512, seed: int = 1004, n_min: int = 32, n_max: int = 96):
    """Recipe of the batch workload: for system i, in order, from numpy's default_rng(seed):
    dimension d uniform in {2, 3}; side N uniform in [n_min, n_max] (N^d interior nodes);
    jump a_hi = 10^U(2, 6); convection components U(0, 30) (d of them); a box (each axis an
    interval with endpoints drawn U(0, 1) and sorted, integer positions over 1000) where
    a = a_hi, a = 1 elsewhere. Returns a list of dicts (no matrices), so sizes and memory can
    be planned before any system is assembled."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        d = int(rng.integers(2, 4))
        N = int(rng.integers(n_min, n_max + 1))
        jump = float(10.0 ** rng.uniform(2.0, 6.0))
        conv = tuple(float(c) for c in rng.uniform(0.0, 30.0, size=d))
        box = [tuple(sorted(int(v) for v in rng.integers(0, 1001, size=2))) for _ in range(d)]
        specs.append({"index": i, "dims": (N,) * d, "jump": jump, "conv": conv, "box": box,
                      "seed": seed})
    return specs


def batch_system(spec) -> Problem:
    """Assemble one batch system from its spec: a = jump inside the box (the open interval of
    each axis, tested exactly with integers: lo/1000 < q/den < hi/1000), 1 elsewhere;
    b = A u* with u* the sine product."""
    d = len(spec["dims"])
    jump = spec["jump"]
    box = spec["box"]

    def diff(q, den):
        inside = np.ones(np.broadcast_shapes(*[x.shape for x in q]), dtype=bool)
        for a in range(d):
            lo, hi = box[a]
            inside &= (1000 * q[a] > lo * den[a]) & (1000 * q[a] < hi * den[a])
        return np.where(inside, jump, 1.0)

    return assemble(spec["dims"], diff, spec["conv"], u_star_fn=_sine_product,
                    name=f"batch_{spec['seed']}_{spec['index']}")


# ---------------------------------------------------------------------------------------
# Small generic systems for unit tests
# ---------------------------------------------------------------------------------------

def laplacian(dims: Sequence[int], conv=None) -> Problem:
    """Constant-coefficient h^2-scaled Laplacian (a = 1), optional constant convection,
    b = A * ones."""
    d = len(dims)
    conv = conv if conv is not None else (0.0,) * d
    return assemble(dims, lambda q, den: np.ones(1), conv, u_star_fn=lambda q, den: np.ones(1),
                    name=f"laplacian_{'x'.join(map(str, dims))}")


def random_sparse(n: int, nnz_per_row: int, seed: int, integer: bool = False,
                  diag_boost: float = 0.0, max_row: Optional[int] = None) -> Problem:
    """Random CSR matrix with sorted, distinct columns in each row; row lengths vary
    between 1 and 2*nnz_per_row (or up to max_row); the diagonal is always present.
    integer=True draws small integers (exact products and sums in FP64)."""
    rng = np.random.default_rng(seed)
    hi = max_row if max_row is not None else 2 * nnz_per_row
    hi = max(1, min(hi, n))
    lens = rng.integers(1, hi + 1, size=n)
    rows = []
    for i in range(n):
        k = int(lens[i])
        others = rng.choice(n - 1, size=k - 1, replace=False) if k > 1 else np.zeros(0, np.int64)
        others = np.where(others >= i, others + 1, others)
        rows.append(np.sort(np.concatenate([others, [i]])))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum([len(r) for r in rows])
    col_idx = np.concatenate(rows).astype(np.int32) if rows else np.zeros(0, np.int32)
    nnz = int(row_ptr[-1])
    if integer:
        val = rng.integers(-8, 9, size=nnz).astype(np.float64)
        val[val == 0] = 1.0
    else:
        val = rng.standard_normal(nnz)
    if diag_boost:
        for i in range(n):
            s, e = row_ptr[i], row_ptr[i + 1]
            j = s + int(np.searchsorted(col_idx[s:e], i))
            val[j] += diag_boost * np.sign(val[j] if val[j] != 0 else 1.0)
    b = rng.integers(-8, 9, size=n).astype(np.float64) if integer else rng.standard_normal(n)
    return Problem(name=f"random_n{n}_s{seed}", dims=(n,), row_ptr=row_ptr.astype(np.int32),
                   col_idx=col_idx, val=val, b=b)
