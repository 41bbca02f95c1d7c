// Batched Bi-CGSTAB and the solve engine: many independent systems share every launch.
//
// Each system is one Bi-CGSTAB solve of section 2 (shadow residual r^ = r0, the stop test of
// section 2.2), exactly as in bicgstab.hip: the same kernels' arithmetic, the same tile
// partition of its rows, the same per-tile partials summed in the same order. A system
// therefore returns bit for bit the result it returns when solved alone with gsk_bicgstab,
// whatever else shares the batch.
//
// Layout. The engine owns a workspace with room for max_rows rows of vectors (r, r^, p x2,
// v x2, t) and max_systems control blocks. A system of n rows gets ceil(n / BS) consecutive
// tiles of that row space (first fit over free tiles); its matrix, b, x and stop weights stay
// in the caller's memory. A device list holds the tiles of the admitted systems (with each
// tile's system); a streaming launch has one workgroup per list entry (the grid rounded up
// to a few sizes, each with its own captured graph), so it costs work only for admitted
// systems; a finalize launch has one workgroup per system slot and sums that
// system's tile partials.
//
// A system may be submitted unscaled with a GS(p) stage (section 2, eq. (2)): the first chunk
// scales its rows into caller-provided outputs (with the arithmetic of gsk_gs_scale) and the
// solve then runs on the scaled system, so GS(p) and Bi-CGSTAB run in the same launches.
//
// Time. The host enqueues chunks: the GS launch (scales newly admitted systems that asked for
// it), the residual launch (starts newly admitted systems and verifies convergence claims),
// then check_every iterations. For a given grid size a chunk has fixed launch shapes and
// arguments, so it can be captured once in a HIP graph and replayed. Between
// chunks the host reads every slot's status and retires finished systems; new systems are
// admitted between chunks (continuous batching).
#include <map>
#include <vector>

#include "batch.hpp"

namespace gsk {

struct BArgsB {
  const SysDesc* sys;
  const int* act;        // [2][max_units]: units of the admitted systems, then their slots
  const int* n_act;      // number of entries in act
  BCtl* ctl;             // [max_systems]
  double* partials;      // [4][max_tiles]
  int max_tiles;
  int max_units;         // list capacity (its second half starts there)
  int rv;                // tiles per list unit (1 or 2)
  double* r;
  double* rh;
  double* p[2];
  double* v[2];
  double* t;
  int par;               // buffer parity of this iteration
};

// Calls body(tile, slot) for the list entry of this workgroup (logical block k takes entry k;
// consecutive entries, adjacent rows of one system, go to one XCD). Workgroups past the end of
// the list (the launch grid is the list length rounded up) return at once.
template <class Body>
__device__ inline void for_active_tiles(const BArgsB& a, Body body) {
  const int k = logical_block();
  if (k >= *a.n_act) return;
  const int unit = a.act[k], s = a.act[a.max_units + k];
  if (a.rv == 1) {
    body(unit, s);
    return;
  }
  // the unit's tiles in turn (the workgroup's LDS is reused between them)
  const int t0 = a.sys[s].tile_off + (unit - a.sys[s].unit_off) * a.rv;
  const int t1 = a.sys[s].tile_off + a.sys[s].ntiles;
  for (int q = 0; q < a.rv && t0 + q < t1; ++q) {
    if (q) __syncthreads();
    body(t0 + q, s);
  }
}

// Calls body(unit, slot) for the list entry of this workgroup (one unit of rv tiles).
template <class Body>
__device__ inline void for_active_units(const BArgsB& a, Body body) {
  const int k = logical_block();
  if (k < *a.n_act) body(a.act[k], a.act[a.max_units + k]);
}

__device__ inline double2 ld2(const double* p) { return *reinterpret_cast<const double2*>(p); }

struct GatherPB {
  const double* __restrict__ r;
  const double* __restrict__ p;
  const double* __restrict__ v;
  double beta, omega;
  int first;
  struct Raw {
    double r, p, v;
  };
  struct Raw2 {   // the operands of rows col and col + 1 (16-byte loads; col even)
    double2 r, p, v;
  };
  __device__ Raw load(int col) const { return Raw{r[col], p[col], v[col]}; }
  __device__ Raw2 load2(int col) const { return Raw2{ld2(r + col), ld2(p + col), ld2(v + col)}; }
  __device__ static Raw half(const Raw2& a, int h) {
    return h ? Raw{a.r.y, a.p.y, a.v.y} : Raw{a.r.x, a.p.x, a.v.x};
  }
  __device__ double value(const Raw& a) const {
    return first ? a.r : fma(beta, fma(-omega, a.v, a.p), a.r);
  }
  __device__ double operator()(int col) const { return value(load(col)); }
};

struct GatherSB {
  const double* __restrict__ r;
  const double* __restrict__ v;
  double alpha;
  struct Raw {
    double r, v;
  };
  struct Raw2 {
    double2 r, v;
  };
  __device__ Raw load(int col) const { return Raw{r[col], v[col]}; }
  __device__ Raw2 load2(int col) const { return Raw2{ld2(r + col), ld2(v + col)}; }
  __device__ static Raw half(const Raw2& a, int h) {
    return h ? Raw{a.r.y, a.v.y} : Raw{a.r.x, a.v.x};
  }
  __device__ double value(const Raw& a) const { return fma(-alpha, a.v, a.r); }
  __device__ double operator()(int col) const { return value(load(col)); }
};

// The system's product over one tile (CSR or stencil, chosen per system).
template <class G>
__device__ inline double sys_tile(const SysDesc& d, int row0, int nrows, const G& g,
                                  TileLds& L) {
  if (d.kind == MAT_STENCIL) {
    EmptyLds e;
    const StencilOp op{d.coef, d.n, d.nx, d.ny, d.nz, (size_t)d.n};
    return op.tile(row0, nrows, g, e);
  }
  const CsrOp op{d.rp, d.ci, d.val};
  return op.tile(row0, nrows, g, L);
}

// The two tiles of a unit (system-local tile lt0 = first) and their rows.
__device__ inline void unit_rows2(const SysDesc& d, int unit, int& lt0, int (&row0)[2],
                                  int (&nr)[2]) {
  lt0 = (unit - d.unit_off) * 2;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    row0[k] = (lt0 + k) * BS;
    nr[k] = max(0, min(BS, d.n - row0[k]));
  }
}

// ---------------------------------------------------------------------------------------
// Stencil units of two tiles through an LDS window.
//
// The gathered value g of every row in [R0 - nx, R0 + 2 BS + nx) (the unit's rows and one
// x-line on either side, clipped to the system) is formed once into LDS; a row then takes its
// -y, -x, centre, +x and +y operands from the window and gathers only -z and +z from global
// memory. Each row is summed in the stencil's position order with the same roundings as
// StencilOp, so the product, the row's own value and every partial equal the global-gather
// form bit for bit.
//
// Pair layout (16-byte loads): with n and nx even and the planes (and stop weights) 16-byte
// aligned, thread t owns rows R0 + 2t and R0 + 2t + 1 and loads coefficients, window entries
// and z-neighbours two rows at a time; the per-row dot-product terms then pass through LDS so
// that each tile's partials are reduced in the single solver's order (row t of the tile in
// thread t). Otherwise thread t owns rows R0 + t and R0 + BS + t (8-byte loads).
// ---------------------------------------------------------------------------------------
constexpr int WIN_NX = 256;                  // widest x-line the window serves
constexpr int WIN_ROWS = 2 * BS + 2 * WIN_NX;

union UnitLds {
  TileLds csr;                               // CSR tiles (one at a time)
  double g[WIN_ROWS];                        // the window of gathered values
  double acc[4][2 * BS];                     // per-row dot-product terms (pair layout)
};

// Positions present in row i's stencil: bit q for -z, -y, -x, centre, +x, +y, +z (as in
// StencilOp).
__device__ inline unsigned stencil_present(const SysDesc& d, int i) {
  const int ix = i % d.nx, rest = i / d.nx, iy = rest % d.ny, iz = rest / d.ny;
  const bool three = d.nz > 1;
  return (three && iz > 0 ? 1u : 0u) | (iy > 0 ? 2u : 0u) | (ix > 0 ? 4u : 0u) | 8u |
         (ix < d.nx - 1 ? 16u : 0u) | (iy < d.ny - 1 ? 32u : 0u) |
         (three && iz < d.nz - 1 ? 64u : 0u);
}

// Coefficient plane of position q (-1: none; the -z and +z positions of a 2D system).
__device__ inline int plane_of(int q, bool three) {
  return three ? q : (q == 0 || q == 6 ? -1 : q - 1);
}

__device__ inline bool unit_pairs(const SysDesc& d, const double* extra) {
  return !(d.n & 1) && !(d.nx & 1) && !(reinterpret_cast<uintptr_t>(d.coef) & 15) &&
         !(reinterpret_cast<uintptr_t>(extra) & 15);
}

// Sum of the row's stencil terms in position order (absent positions add +0.0).
__device__ inline double stencil_sum(unsigned present, const double (&c)[7],
                                     const double (&g)[7]) {
#pragma clang fp contract(off)
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < 7; ++q) s += (present >> q) & 1u ? c[q] * g[q] : 0.0;
  return s;
}

// y[h] = (A g)_row[h] and gv[h] = g(row[h]) for the thread's two row slots of the unit's rows
// [R0, R0 + nr) of system d (stencil, nx <= WIN_NX); ok[h]: the slot is a row of the unit.
// pair: slots are rows R0 + 2t and R0 + 2t + 1 (requires unit_pairs), else R0 + t and
// R0 + BS + t. All threads of the workgroup call (one barrier); gw is the LDS window.
template <class G>
__device__ inline void unit_window(const SysDesc& d, int R0, int nr, bool pair, const G& g,
                                   double* gw, int (&row)[2], bool (&ok)[2], double (&y)[2],
                                   double (&gv)[2]) {
  const int t = threadIdx.x;
  const int n = d.n, nx = d.nx;
  const int nxy = nx * d.ny;
  const bool three = d.nz > 1;
  const int W0 = max(0, R0 - nx);
  const int W1 = min(n, R0 + 2 * BS + nx);
  const int wn = W1 - W0;
  double c[2][7];
  if (pair) {
    row[0] = R0 + min(2 * t, nr - 2);
    row[1] = row[0] + 1;
    ok[0] = ok[1] = 2 * t < nr;
    const int wp = wn >> 1;
    typename G::Raw2 f[WIN_ROWS / (2 * BS)];
#pragma unroll
    for (int q = 0; q < WIN_ROWS / (2 * BS); ++q)
      f[q] = g.load2(W0 + 2 * min(q * BS + t, wp - 1));
#pragma unroll
    for (int q = 0; q < 7; ++q) {
      const int pl = plane_of(q, three);
      const double2 cc = pl >= 0 ? ld2(d.coef + (size_t)pl * n + row[0]) : double2{0.0, 0.0};
      c[0][q] = cc.x;
      c[1][q] = cc.y;
    }
    typename G::Raw2 z[2];
    z[0] = g.load2(max(row[0] - nxy, 0));
    z[1] = g.load2(min(row[0] + nxy, n - 2));
#pragma unroll
    for (int q = 0; q < WIN_ROWS / (2 * BS); ++q) {
      const int kk = q * BS + t;
      if (kk < wp) {
        gw[2 * kk] = g.value(G::half(f[q], 0));
        gw[2 * kk + 1] = g.value(G::half(f[q], 1));
      }
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int li = row[h] - W0;
      double gq[7];
      gq[0] = three ? g.value(G::half(z[0], h)) : 0.0;
      gq[1] = gw[max(li - nx, 0)];
      gq[2] = gw[max(li - 1, 0)];
      gq[3] = gw[li];
      gq[4] = gw[min(li + 1, wn - 1)];
      gq[5] = gw[min(li + nx, wn - 1)];
      gq[6] = three ? g.value(G::half(z[1], h)) : 0.0;
      y[h] = stencil_sum(stencil_present(d, row[h]), c[h], gq);
      gv[h] = gq[3];
    }
  } else {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      row[h] = R0 + min(h * BS + t, nr - 1);
      ok[h] = h * BS + t < nr;
    }
    typename G::Raw f[WIN_ROWS / BS];
#pragma unroll
    for (int q = 0; q < WIN_ROWS / BS; ++q)
      if (q * BS < wn) f[q] = g.load(W0 + min(q * BS + t, wn - 1));
    typename G::Raw z[2][2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int q = 0; q < 7; ++q) {
        const int pl = plane_of(q, three);
        c[h][q] = pl >= 0 ? d.coef[(size_t)pl * n + row[h]] : 0.0;
      }
      z[h][0] = g.load(max(row[h] - nxy, 0));
      z[h][1] = g.load(min(row[h] + nxy, n - 1));
    }
#pragma unroll
    for (int q = 0; q < WIN_ROWS / BS; ++q) {
      const int kk = q * BS + t;
      if (q * BS < wn && kk < wn) gw[kk] = g.value(f[q]);
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int li = row[h] - W0;
      double gq[7];
      gq[0] = three ? g.value(z[h][0]) : 0.0;
      gq[1] = gw[max(li - nx, 0)];
      gq[2] = gw[max(li - 1, 0)];
      gq[3] = gw[li];
      gq[4] = gw[min(li + 1, wn - 1)];
      gq[5] = gw[min(li + nx, wn - 1)];
      gq[6] = three ? g.value(z[h][1]) : 0.0;
      y[h] = stencil_sum(stencil_present(d, row[h]), c[h], gq);
      gv[h] = gq[3];
    }
  }
}

// Partials of NC per-row terms of the unit's two tiles (tile k holds unit rows
// [k BS, (k+1) BS)), each tile reduced in the single solver's order: row t of the tile in
// thread t. In the pair layout the terms pass through the LDS acc array (which may alias the
// window: the caller has finished reading it). `tiles` = tiles of the unit inside the system.
template <int NC>
__device__ inline void unit_partials(bool pair, const double (&acc)[2][NC], double (*lds)[2 * BS],
                                     int tiles, double* partials, int stride, int tile0,
                                     double* red) {
  const int t = threadIdx.x;
  double v[2][NC];
  if (pair) {
    __syncthreads();   // the window is no longer read
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int c = 0; c < NC; ++c) lds[c][2 * t + h] = acc[h][c];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int c = 0; c < NC; ++c) v[k][c] = lds[c][k * BS + t];
  } else {
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int c = 0; c < NC; ++c) v[k][c] = acc[k][c];
  }
  for (int k = 0; k < tiles; ++k) {
    if (k) __syncthreads();
    block_partials<NC>(v[k], NC, partials, stride, tile0 + k, red);
  }
}

__global__ __launch_bounds__(64) void k_batch_init(BCtl* c, int maxit, double tol, double eps_b,
                                                   int has_w, int scale) {
  if (threadIdx.x != 0) return;
  c->sum.state = scale ? ST_SCALE : ST_INIT;
  c->sum.status = S_MAXIT;
  c->sum.iters = 0;
  c->sum.restarts = 0;
  c->sum.half = 0;
  c->sum.fails = 0;
  c->sum.steps = 0;
  c->sum.relres_rec = 1.0;
  c->sum.relres_true = 1.0;
  c->sum.brk = BRK_NONE;
  c->maxit = maxit;
  c->first = 1;
  c->has_w = has_w;
  c->bad = 0;
  c->tol = tol;
  c->eps_b = eps_b;
  c->ref = 0.0;
  c->rho = c->rho_old = c->alpha = c->omega = c->beta = c->rh_norm = 0.0;
  c->target = tol;
  c->last_rt = 1.0;
}

// Flat validity scan of one system's CSR structure (no indirect loads): row_ptr[0] == 0,
// non-decreasing, row_ptr[n] == nnz, every column index in [0, n). Sets BAD_CSR in *bad_bits.
__global__ __launch_bounds__(BS) void k_batch_validate(const int* __restrict__ rp,
                                                       const int* __restrict__ ci, int n,
                                                       int64_t nnz, int* bad_bits) {
  const int64_t stride = (int64_t)gridDim.x * BS;
  const int64_t gid = (int64_t)blockIdx.x * BS + threadIdx.x;
  bool bad = false;
  for (int64_t i = gid; i <= n; i += stride) {
    const int r = rp[i];
    if (i == 0 && r != 0) bad = true;
    if (i < n && r > rp[i + 1]) bad = true;
    if (i == n && (int64_t)r != nnz) bad = true;
  }
  for (int64_t k = gid; k < nnz; k += stride) {
    const int col = ci[k];
    if (col < 0 || col >= n) bad = true;
  }
  if (bad) atomicOr(bad_bits, BAD_CSR);
}

// G: GS(p) of the systems whose stage is pending (same arithmetic as k_gs_scale).
__global__ __launch_bounds__(BS) void k_batch_gs(BArgsB a) {
  __shared__ GsLds L;
  for_active_tiles(a, [&](int tile, int s) {
    const SysDesc d = a.sys[s];
    BCtl* c = a.ctl + s;
    if (c->sum.state != ST_SCALE || (c->bad & BAD_CSR)) return;
    prepare_tile(d, tile - d.tile_off, L, &c->bad);
  });
}

__global__ __launch_bounds__(64) void k_batch_fin_gs(BArgsB a) {
  const int s = blockIdx.x;
  if (threadIdx.x != 0 || a.sys[s].ntiles == 0) return;
  BCtl* c = a.ctl + s;
  if (c->sum.state != ST_SCALE) return;
  c->sum.state = ST_INIT;   // a GS error (c->bad) is reported by the residual stage
}

// R: r = b - A x, r^ = r for systems starting, verifying or finishing; ||r||^2, ||W r||^2.
__global__ __launch_bounds__(BS) void k_batch_residual(BArgsB a) {
  __shared__ TileLds L;
  __shared__ double red[NC_MAX * WAVES];
  for_active_tiles(a, [&](int tile, int s) {
    const SysDesc d = a.sys[s];
    BCtl* c = a.ctl + s;
    const int st = c->sum.state;
    if (st != ST_INIT && st != ST_VERIFY && st != ST_FINAL) return;
    if (c->bad) return;
    const int row0 = (tile - d.tile_off) * BS;
    const int nrows = min(BS, d.n - row0);
    const int t = threadIdx.x;
    double acc[2] = {0.0, 0.0};
    const double y = sys_tile(d, row0, nrows, GatherX{d.x}, L);
    if (t < nrows) {
      const int row = row0 + t;
      const double r = d.b[row] - y;
      if (st != ST_FINAL) {
        a.r[d.row_off + row] = r;
        a.rh[d.row_off + row] = r;
      }
      acc[0] = r * r;
      if (d.W) {
        const double wr = d.W[row] * r;
        acc[1] = wr * wr;
      }
    }
    block_partials<2>(acc, 2, a.partials, a.max_tiles, tile, red);
  });
}

__global__ __launch_bounds__(BS) void k_batch_fin_residual(BArgsB a) {
  const int s = blockIdx.x;
  const SysDesc d = a.sys[s];
  if (d.ntiles == 0) return;
  BCtl* c = a.ctl + s;
  const int st = c->sum.state;
  if (st != ST_INIT && st != ST_VERIFY && st != ST_FINAL) return;
  if (c->bad) {
    if (threadIdx.x == 0) {
      c->sum.state = ST_DONE;
      c->sum.status = bad_status(c->bad);
    }
    return;
  }
  __shared__ double out[8];
  small_sums_strided<2>(a.partials + d.tile_off, d.ntiles, a.max_tiles, out);
  if (threadIdx.x != 0) return;
  const double nr = sqrt(out[0]);
  const double nwr = d.W ? sqrt(out[1]) : nr;
  if (st == ST_INIT) {
    c->ref = nwr;
    if (nwr == 0.0) {
      c->sum.status = S_CONVERGED;
      c->sum.relres_rec = 0.0;
      c->sum.relres_true = 0.0;
      c->sum.state = ST_DONE;
      return;
    }
    if (c->maxit == 0) {
      c->sum.status = S_MAXIT;
      c->sum.state = ST_DONE;
      return;
    }
  } else {
    const double rt = nwr / c->ref;
    c->sum.relres_true = rt;
    if (st == ST_FINAL) {
      c->sum.state = ST_DONE;
      return;
    }
    if (rt < c->tol) {
      c->sum.status = S_CONVERGED;
      c->sum.state = ST_DONE;
      return;
    }
    if (c->sum.iters >= c->maxit) {
      c->sum.status = S_MAXIT;
      c->sum.state = ST_DONE;
      return;
    }
    c->sum.fails += 1;
    if (c->sum.fails >= 3) {
      c->sum.status = S_STAGNATED;
      c->sum.state = ST_DONE;
      return;
    }
    c->sum.restarts += 1;
  }
  c->rh_norm = nr;
  c->rho = out[0];
  c->sum.half = 0;
  if (fabs(c->rho) <= c->eps_b * nr * nr) {
    c->sum.status = S_BREAKDOWN;
    c->sum.brk = BRK_RHO;
    c->sum.state = ST_DONE;
    return;
  }
  c->first = 1;
  c->sum.state = ST_RUNNING;
}

// P: new p, v = A p; partials (r^, v), ||v||^2.
template <int RV>
__global__ __launch_bounds__(BS) void k_batch_p(BArgsB a) {
  __shared__ UnitLds U;
  TileLds& L = U.csr;
  __shared__ double red[NC_MAX * WAVES];
  if constexpr (RV == 1) {
    for_active_tiles(a, [&](int tile, int s) {
      const SysDesc d = a.sys[s];
      BCtl* c = a.ctl + s;
      if (c->sum.state != ST_RUNNING) return;
      const int q = a.par;
      const int64_t o = d.row_off;
      const GatherPB G{a.r + o, a.p[q] + o, a.v[q] + o, c->beta, c->omega, c->first};
      const int row0 = (tile - d.tile_off) * BS;
      const int nrows = min(BS, d.n - row0);
      const int t = threadIdx.x;
      const double y = sys_tile(d, row0, nrows, G, L);
      double acc[2] = {0.0, 0.0};
      if (t < nrows) {
        const int row = row0 + t;
        a.p[q ^ 1][o + row] = G(row);
        a.v[q ^ 1][o + row] = y;
        acc[0] = a.rh[o + row] * y;
        acc[1] = y * y;
      }
      block_partials<2>(acc, 2, a.partials, a.max_tiles, tile, red);
    });
  } else {
    // two tiles per workgroup: a stencil product loads both tiles' operands before either
    // sum; partials stay per tile
    for_active_units(a, [&](int unit, int s) {
      const SysDesc d = a.sys[s];
      BCtl* c = a.ctl + s;
      if (c->sum.state != ST_RUNNING) return;
      const int q = a.par;
      const int64_t o = d.row_off;
      const GatherPB G{a.r + o, a.p[q] + o, a.v[q] + o, c->beta, c->omega, c->first};
      int lt0, row0[2], nr[2];
      unit_rows2(d, unit, lt0, row0, nr);
      if (d.kind == MAT_STENCIL && d.nx <= WIN_NX) {
        const bool pair = unit_pairs(d, nullptr);
        const int R0 = row0[0], nu = nr[0] + nr[1];
        int row[2];
        bool ok[2];
        double y[2], gv[2];
        unit_window(d, R0, nu, pair, G, U.g, row, ok, y, gv);
        double acc[2][2];
        double rh[2];
        if (pair) {
          const double2 r2 = ld2(a.rh + o + row[0]);
          rh[0] = r2.x;
          rh[1] = r2.y;
        } else {
          rh[0] = a.rh[o + row[0]];
          rh[1] = a.rh[o + row[1]];
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          acc[h][0] = ok[h] ? rh[h] * y[h] : 0.0;
          acc[h][1] = ok[h] ? y[h] * y[h] : 0.0;
        }
        if (pair) {
          if (ok[0]) {
            *reinterpret_cast<double2*>(a.p[q ^ 1] + o + row[0]) = double2{gv[0], gv[1]};
            *reinterpret_cast<double2*>(a.v[q ^ 1] + o + row[0]) = double2{y[0], y[1]};
          }
        } else {
#pragma unroll
          for (int h = 0; h < 2; ++h)
            if (ok[h]) {
              a.p[q ^ 1][o + row[h]] = gv[h];
              a.v[q ^ 1][o + row[h]] = y[h];
            }
        }
        unit_partials<2>(pair, acc, U.acc, nr[1] > 0 ? 2 : 1, a.partials, a.max_tiles,
                         d.tile_off + lt0, red);
        return;
      }
      // CSR, or x-lines wider than the window: one tile at a time
      const int t = threadIdx.x;
      for (int k = 0; k < 2; ++k) {
        if (nr[k] <= 0) break;
        if (k) __syncthreads();
        const double y = sys_tile(d, row0[k], nr[k], G, L);
        double acc[2] = {0.0, 0.0};
        if (t < nr[k]) {
          const int row = row0[k] + t;
          a.p[q ^ 1][o + row] = G(row);
          a.v[q ^ 1][o + row] = y;
          acc[0] = a.rh[o + row] * y;
          acc[1] = y * y;
        }
        block_partials<2>(acc, 2, a.partials, a.max_tiles, d.tile_off + lt0 + k, red);
      }
    });
  }
}

__global__ __launch_bounds__(BS) void k_batch_fin_p(BArgsB a) {
  const int s = blockIdx.x;
  const SysDesc d = a.sys[s];
  if (d.ntiles == 0) return;
  BCtl* c = a.ctl + s;
  if (c->sum.state != ST_RUNNING) return;
  __shared__ double out[8];
  small_sums_strided<2>(a.partials + d.tile_off, d.ntiles, a.max_tiles, out);
  if (threadIdx.x != 0) return;
  const double sigma = out[0];
  const double vn = sqrt(out[1]);
  if (fabs(sigma) <= c->eps_b * c->rh_norm * vn) {
    c->sum.status = S_BREAKDOWN;
    c->sum.brk = BRK_SIGMA;
    c->sum.state = ST_FINAL;
    return;
  }
  c->alpha = c->rho / sigma;
}

// S: t = A s with s = r - alpha v; partials (t,s), (t,t), ||s||^2, ||W s||^2.
template <int RV>
__global__ __launch_bounds__(BS) void k_batch_s(BArgsB a) {
  __shared__ UnitLds U;
  TileLds& L = U.csr;
  __shared__ double red[NC_MAX * WAVES];
  if constexpr (RV == 1) {
    for_active_tiles(a, [&](int tile, int s) {
      const SysDesc d = a.sys[s];
      BCtl* c = a.ctl + s;
      if (c->sum.state != ST_RUNNING) return;
      const int64_t o = d.row_off;
      const GatherSB G{a.r + o, a.v[a.par ^ 1] + o, c->alpha};
      const int row0 = (tile - d.tile_off) * BS;
      const int nrows = min(BS, d.n - row0);
      const int t = threadIdx.x;
      const double y = sys_tile(d, row0, nrows, G, L);
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      if (t < nrows) {
        const int row = row0 + t;
        const double sv = G(row);
        a.t[o + row] = y;
        acc[0] = y * sv;
        acc[1] = y * y;
        acc[2] = sv * sv;
        if (d.W) {
          const double ws = d.W[row] * sv;
          acc[3] = ws * ws;
        }
      }
      block_partials<4>(acc, 4, a.partials, a.max_tiles, tile, red);
    });
  } else {
    for_active_units(a, [&](int unit, int s) {
      const SysDesc d = a.sys[s];
      BCtl* c = a.ctl + s;
      if (c->sum.state != ST_RUNNING) return;
      const int64_t o = d.row_off;
      const GatherSB G{a.r + o, a.v[a.par ^ 1] + o, c->alpha};
      int lt0, row0[2], nr[2];
      unit_rows2(d, unit, lt0, row0, nr);
      if (d.kind == MAT_STENCIL && d.nx <= WIN_NX) {
        const bool pair = unit_pairs(d, d.W);
        const int R0 = row0[0], nu = nr[0] + nr[1];
        int row[2];
        bool ok[2];
        double y[2], sv[2];
        unit_window(d, R0, nu, pair, G, U.g, row, ok, y, sv);
        double wv[2] = {0.0, 0.0};
        if (d.W) {
          if (pair) {
            const double2 w2 = ld2(d.W + row[0]);
            wv[0] = w2.x;
            wv[1] = w2.y;
          } else {
            wv[0] = d.W[row[0]];
            wv[1] = d.W[row[1]];
          }
        }
        double acc[2][4];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          acc[h][0] = ok[h] ? y[h] * sv[h] : 0.0;
          acc[h][1] = ok[h] ? y[h] * y[h] : 0.0;
          acc[h][2] = ok[h] ? sv[h] * sv[h] : 0.0;
          const double ws = wv[h] * sv[h];
          acc[h][3] = ok[h] && d.W ? ws * ws : 0.0;
        }
        if (pair) {
          if (ok[0]) *reinterpret_cast<double2*>(a.t + o + row[0]) = double2{y[0], y[1]};
        } else {
#pragma unroll
          for (int h = 0; h < 2; ++h)
            if (ok[h]) a.t[o + row[h]] = y[h];
        }
        unit_partials<4>(pair, acc, U.acc, nr[1] > 0 ? 2 : 1, a.partials, a.max_tiles,
                         d.tile_off + lt0, red);
        return;
      }
      // CSR, or x-lines wider than the window: one tile at a time
      const int t = threadIdx.x;
      for (int k = 0; k < 2; ++k) {
        if (nr[k] <= 0) break;
        if (k) __syncthreads();
        const double y = sys_tile(d, row0[k], nr[k], G, L);
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        if (t < nr[k]) {
          const int row = row0[k] + t;
          const double sv = G(row);
          a.t[o + row] = y;
          acc[0] = y * sv;
          acc[1] = y * y;
          acc[2] = sv * sv;
          if (d.W) {
            const double ws = d.W[row] * sv;
            acc[3] = ws * ws;
          }
        }
        block_partials<4>(acc, 4, a.partials, a.max_tiles, d.tile_off + lt0 + k, red);
      }
    });
  }
}

__global__ __launch_bounds__(BS) void k_batch_fin_s(BArgsB a) {
  const int s = blockIdx.x;
  const SysDesc d = a.sys[s];
  if (d.ntiles == 0) return;
  BCtl* c = a.ctl + s;
  if (c->sum.state != ST_RUNNING) return;
  __shared__ double out[8];
  small_sums_strided<4>(a.partials + d.tile_off, d.ntiles, a.max_tiles, out);
  if (threadIdx.x != 0) return;
  c->sum.iters += 1;
  const double sn = sqrt(out[2]);
  const double est = (d.W ? sqrt(out[3]) : sn) / c->ref;
  c->sum.relres_rec = est;
  if (est < c->tol) {
    c->sum.half = 1;
    c->sum.state = ST_HALF;
    return;
  }
  const double ts = out[0], tt = out[1];
  if (fabs(ts) <= c->eps_b * sqrt(tt) * sn) {
    c->sum.status = S_BREAKDOWN;
    c->sum.brk = BRK_OMEGA;
    c->sum.state = ST_FINAL;
    return;
  }
  c->omega = ts / tt;
}

// U: x += alpha p + omega s, r = s - omega t; partials (r^, r), ||r||^2, ||W r||^2.
// After a half-step exit only x += alpha p is done.
__global__ __launch_bounds__(BS) void k_batch_u(BArgsB a) {
  __shared__ double red[NC_MAX * WAVES];
  for_active_tiles(a, [&](int tile, int s) {
    const SysDesc d = a.sys[s];
    BCtl* c = a.ctl + s;
    const int st = c->sum.state;
    if (st != ST_RUNNING && st != ST_HALF) return;
    const int q = a.par ^ 1;
    const int64_t o = d.row_off;
    const double* p = a.p[q] + o;
    const double* v = a.v[q] + o;
    const double alpha = c->alpha, omega = c->omega;
    const int row = (tile - d.tile_off) * BS + threadIdx.x;
    const bool mine = row < d.n;
    if (st == ST_HALF) {
      if (mine) d.x[row] = fma(alpha, p[row], d.x[row]);
      return;
    }
    double acc[3] = {0.0, 0.0, 0.0};
    if (mine) {
      const double sv = fma(-alpha, v[row], a.r[o + row]);
      d.x[row] = fma(omega, sv, fma(alpha, p[row], d.x[row]));
      const double r = fma(-omega, a.t[o + row], sv);
      a.r[o + row] = r;
      acc[0] = a.rh[o + row] * r;
      acc[1] = r * r;
      if (d.W) {
        const double wr = d.W[row] * r;
        acc[2] = wr * wr;
      }
    }
    block_partials<3>(acc, 3, a.partials, a.max_tiles, tile, red);
  });
}

__global__ __launch_bounds__(BS) void k_batch_fin_u(BArgsB a) {
  const int s = blockIdx.x;
  const SysDesc d = a.sys[s];
  if (d.ntiles == 0) return;
  BCtl* c = a.ctl + s;
  const int st = c->sum.state;
  if (st != ST_RUNNING && st != ST_HALF) return;
  if (st == ST_HALF) {
    if (threadIdx.x == 0) c->sum.state = ST_VERIFY;
    return;
  }
  __shared__ double out[8];
  small_sums_strided<3>(a.partials + d.tile_off, d.ntiles, a.max_tiles, out);
  if (threadIdx.x != 0) return;
  const double rn = sqrt(out[1]);
  const double est = (d.W ? sqrt(out[2]) : rn) / c->ref;
  c->sum.relres_rec = est;
  if (est < c->tol || c->sum.iters >= c->maxit) {
    c->sum.state = ST_VERIFY;
    return;
  }
  const double rho_new = out[0];
  if (fabs(rho_new) <= c->eps_b * c->rh_norm * rn) {
    c->sum.status = S_BREAKDOWN;
    c->sum.brk = BRK_RHO;
    c->sum.state = ST_FINAL;
    return;
  }
  c->beta = (rho_new / c->rho) * (c->alpha / c->omega);
  c->rho_old = c->rho;
  c->rho = rho_new;
  c->first = 0;
}

// Measurement: the algorithmic bytes of the launch of class kc that ran just before (per
// system at that stage, the figures of the kernel-class table in gsk.h), into ps->bytes[slot].
// Runs between that launch and its finalize, so every system is in the state the launch saw.
__global__ __launch_bounds__(BS) void k_batch_probe_bytes(BArgsB a, int max_sys, int kc,
                                                          int slot, ProbeSlots* ps) {
  __shared__ double red[NC_MAX * WAVES];
  double acc[1] = {0.0};
  for (int s = threadIdx.x; s < max_sys; s += BS) {
    const SysDesc d = a.sys[s];
    if (d.ntiles == 0) continue;
    const BCtl* c = a.ctl + s;
    const int st = c->sum.state;
    const double n = (double)d.n;
    if (kc == KC_BATCH_U) {
      if (st == ST_RUNNING) acc[0] += (d.W ? 72.0 : 64.0) * n;
      if (st == ST_HALF) acc[0] += 24.0 * n;
      continue;
    }
    if (st != ST_RUNNING) continue;
    // matrix term (a running system's CSR structure has been validated)
    const double M = d.kind == MAT_STENCIL ? 8.0 * (d.nz > 1 ? 7 : 5) * n
                                           : 12.0 * (double)d.rp[d.n] + 4.0 * (n + 1.0);
    if (kc == KC_BATCH_P) acc[0] += M + (c->first ? 32.0 : 48.0) * n;
    if (kc == KC_BATCH_S) acc[0] += M + (d.W ? 32.0 : 24.0) * n;
  }
  block_partials<1>(acc, 1, ps->bytes, 0, slot, red);
}

// ---------------------------------------------------------------------------------------
// Host side: the engine.
// ---------------------------------------------------------------------------------------
constexpr int kBatchVectors = 7;

struct EngineLayout {
  size_t sys, tiles, probe, ctl, sums, partials, vecs, total;
};

static int units_of(const EngineConfig& cfg) {
  if (cfg.mixed) return 2;
  return cfg.method == 0 && cfg.units == 2 ? 2 : 1;   // FP64 Bi-CGSTAB may take two
}

// Workspace carve-up. Bi-CGSTAB: system table, unit list, control blocks, partials (4 per
// tile), the 7 vectors. GMRES: system table, unit list, control blocks, status copies,
// partials (max(m+1, 3) columns per tile and one more for C), basis (m+1 columns) and w, in
// FP64 or FP32.
static EngineLayout engine_layout(const EngineConfig& cfg) {
  const int64_t max_tiles = (cfg.max_rows + BS - 1) / BS;
  const int64_t grid_tiles = (max_tiles + 7) / 8 * 8;
  const size_t ns = (size_t)cfg.max_sys;
  EngineLayout L;
  size_t off = 0;
  L.sys = off;
  off += align256(sizeof(SysDesc) * ns);
  L.tiles = off;
  off += align256(sizeof(int) * (2 * (size_t)grid_tiles + 1));
  L.probe = off;
  off += align256(sizeof(ProbeSlots));
  L.ctl = off;
  if (cfg.method == 1) {
    off += align256(sizeof(Ctl) * ns);
    L.sums = off;
    off += align256(sizeof(Summary) * ns);
    L.partials = off;
    off += align256(sizeof(double) * (size_t)gmres_partial_cols(cfg.m) * (size_t)grid_tiles);
    L.vecs = off;
    const size_t tb = cfg.mixed ? sizeof(float) : sizeof(double);
    off += align256(tb * (size_t)grid_tiles * BS * (size_t)(cfg.m + 1));
    off += align256(tb * (size_t)grid_tiles * BS);
  } else {
    off += align256(sizeof(BCtl) * ns);
    L.sums = off;
    L.partials = off;
    off += align256(sizeof(double) * 4 * (size_t)grid_tiles);
    L.vecs = off;
    off += (size_t)kBatchVectors * align256(sizeof(double) * (size_t)grid_tiles * BS);
  }
  L.total = off;
  return L;
}

size_t engine_workspace_bytes(const EngineConfig& cfg) {
  if (cfg.max_rows < 1 || cfg.max_sys < 1) return 0;
  if (cfg.method == 1 && (cfg.m < 1 || cfg.m > MMAX)) return 0;
  return engine_layout(cfg).total;
}

struct Engine {
  hipStream_t s = nullptr;
  int64_t max_rows = 0;
  int max_sys = 0, max_tiles = 0, grid_tiles = 0, check_every = 8;
  bool use_graph = false;
  int method = 0;                  // 0 Bi-CGSTAB, 1 GMRES(m)
  int m = 0;
  bool mixed = false;
  int rv = 1;                      // tiles per unit
  int max_units = 0;
  bool column = true;              // GMRES basis fits one buffer descriptor
  BArgsB args{};
  GArgs gargs{};
  MArgs margs{};
  SysDesc* d_sys = nullptr;        // device system table and unit list (any method)
  int* d_list = nullptr;
  ProbeSlots* d_probe = nullptr;   // measurement slots (FP64 Bi-CGSTAB engine)
  long long probe_chunks = 0;      // chunks run while a batch kernel class is probed
  bool probe_pending = false;      // timed launches wait for their collection at the next poll
  // host state
  std::vector<SysDesc> h_sys;
  std::vector<int64_t> tags;
  std::vector<char> active;
  std::vector<int> tile_sys;       // slot of every tile, -1 if free
  std::map<int, int> free_tiles;   // start -> length
  bool dirty = true;
  int64_t launched = 0;
  // pinned staging and status
  SysDesc* p_sys = nullptr;
  int* p_tiles = nullptr;
  BCtl* p_ctl = nullptr;
  Summary* p_sums = nullptr;
  hipEvent_t ev_upload = nullptr, ev_chunk = nullptr;
  bool upload_pending = false, chunk_pending = false;
  int n_listed = 0;                          // entries of the device tile list
  std::map<int, hipGraphExec_t> graphs;      // captured chunk per streaming grid size
};

static const Summary& status_of(const Engine& e, int slot) {
  return e.method == 1 ? e.p_sums[slot] : e.p_ctl[slot].sum;
}

// Streaming grid for a list of n tiles: n rounded up to a multiple of 8 (the XCD mapping of
// logical_block needs it) and, from 32 on, to two significant bits (4..7 times a power of two),
// so that the grid, and the captured graph that holds it, changes only when the list has grown
// or shrunk by about a quarter; the surplus workgroups exit at once.
static int stream_grid(int n) {
  int g = n < 8 ? 8 : (n + 7) / 8 * 8;
  int top = 1;
  while (top * 2 <= g) top *= 2;
  if (top >= 32) {
    const int step = top / 4;
    g = (g + step - 1) / step * step;
  }
  return g;
}

static bool alloc_tiles(Engine& e, int need, int& start) {
  for (auto it = e.free_tiles.begin(); it != e.free_tiles.end(); ++it) {
    if (it->second >= need) {
      start = it->first;
      const int rest = it->second - need;
      e.free_tiles.erase(it);
      if (rest > 0) e.free_tiles[start + need] = rest;
      return true;
    }
  }
  return false;
}

static void free_tiles_range(Engine& e, int start, int len) {
  auto it = e.free_tiles.emplace(start, len).first;
  auto next = std::next(it);
  if (next != e.free_tiles.end() && it->first + it->second == next->first) {
    it->second += next->second;
    e.free_tiles.erase(next);
  }
  if (it != e.free_tiles.begin()) {
    auto prev = std::prev(it);
    if (prev->first + prev->second == it->first) {
      prev->second += it->second;
      e.free_tiles.erase(it);
    }
  }
}

int engine_create(void* ws, size_t ws_bytes, const EngineConfig& cfg, hipStream_t s,
                  Engine** out) {
  if (cfg.max_rows < 1 || cfg.max_sys < 1) return -1;
  if (cfg.method == 1 && (cfg.m < 1 || cfg.m > MMAX)) return -1;
  const EngineLayout L = engine_layout(cfg);
  if (ws_bytes < L.total) return -4;
  if (cfg.use_graph && (s == nullptr || (cfg.method == 0 && (cfg.check_every & 1)))) return -1;
  Engine* e = new Engine();
  e->s = s;
  e->max_rows = cfg.max_rows;
  e->max_sys = cfg.max_sys;
  e->max_tiles = (int)((cfg.max_rows + BS - 1) / BS);
  e->grid_tiles = (e->max_tiles + 7) / 8 * 8;
  e->check_every = cfg.check_every;
  e->use_graph = cfg.use_graph;
  e->method = cfg.method;
  e->m = cfg.m;
  e->mixed = cfg.mixed;
  e->rv = units_of(cfg);
  e->max_units = e->grid_tiles / e->rv;
  const int max_sys = cfg.max_sys;
  char* base = static_cast<char*>(ws);
  if (e->method == 1) {
    GArgs& g = e->gargs;
    g.sys = reinterpret_cast<const SysDesc*>(base + L.sys);
    g.act = reinterpret_cast<const int*>(base + L.tiles);
    g.n_act = g.act + 2 * (size_t)e->max_units;
    g.ctl = reinterpret_cast<Ctl*>(base + L.ctl);
    g.sums = reinterpret_cast<Summary*>(base + L.sums);
    g.partials = reinterpret_cast<double*>(base + L.partials);
    g.pstride = e->grid_tiles;
    g.ccol = gmres_partial_cols(cfg.m) - 1;
    g.max_units = e->max_units;
    g.ldv = (size_t)e->grid_tiles * BS;
    const size_t tb = e->mixed ? sizeof(float) : sizeof(double);
    g.V = base + L.vecs;
    g.w = base + L.vecs + align256(tb * g.ldv * (size_t)(cfg.m + 1));
    g.zero = 0.0;
    g.mixed = e->mixed ? 1 : 0;
    e->column = e->mixed ? fits_buffer<float>(g.ldv, cfg.m + 1)
                         : fits_buffer<double>(g.ldv, cfg.m + 1);
  } else if (e->mixed) {
    MArgs& a = e->margs;
    a.sys = reinterpret_cast<const SysDesc*>(base + L.sys);
    a.act = reinterpret_cast<const int*>(base + L.tiles);
    a.n_act = a.act + 2 * (size_t)e->max_units;
    a.ctl = reinterpret_cast<BCtl*>(base + L.ctl);
    a.partials = reinterpret_cast<double*>(base + L.partials);
    a.pstride = e->grid_tiles;
    a.max_units = e->max_units;
    const size_t vb = align256(sizeof(double) * (size_t)e->grid_tiles * BS);
    float* v[kBatchVectors];
    for (int i = 0; i < kBatchVectors; ++i) v[i] = reinterpret_cast<float*>(base + L.vecs + i * vb);
    a.r = v[0];
    a.rh = v[1];
    a.p[0] = v[2];
    a.p[1] = v[3];
    a.v[0] = v[4];
    a.v[1] = v[5];
    a.t = v[6];
    a.delta = cfg.delta;
    a.par = 0;
    e->args.ctl = a.ctl;   // status read-back
  } else {
    BArgsB& a = e->args;
    a.sys = reinterpret_cast<const SysDesc*>(base + L.sys);
    a.act = reinterpret_cast<const int*>(base + L.tiles);
    a.ctl = reinterpret_cast<BCtl*>(base + L.ctl);
    a.partials = reinterpret_cast<double*>(base + L.partials);
    a.max_tiles = e->grid_tiles;
    a.max_units = e->max_units;
    a.rv = e->rv;
    a.n_act = a.act + 2 * (size_t)e->max_units;
    const size_t vb = align256(sizeof(double) * (size_t)e->grid_tiles * BS);
    double* v[kBatchVectors];
    for (int i = 0; i < kBatchVectors; ++i)
      v[i] = reinterpret_cast<double*>(base + L.vecs + i * vb);
    a.r = v[0];
    a.rh = v[1];
    a.p[0] = v[2];
    a.p[1] = v[3];
    a.v[0] = v[4];
    a.v[1] = v[5];
    a.t = v[6];
    a.par = 0;
  }
  e->d_sys = reinterpret_cast<SysDesc*>(base + L.sys);
  e->d_list = reinterpret_cast<int*>(base + L.tiles);
  e->d_probe = reinterpret_cast<ProbeSlots*>(base + L.probe);
  e->h_sys.assign(max_sys, SysDesc{});
  e->tags.assign(max_sys, 0);
  e->active.assign(max_sys, 0);
  e->tile_sys.assign(e->grid_tiles, -1);
  e->free_tiles[0] = e->max_tiles;
  bool ok = hipHostMalloc((void**)&e->p_sys, sizeof(SysDesc) * max_sys, hipHostMallocDefault) ==
                hipSuccess &&
            hipHostMalloc((void**)&e->p_tiles, sizeof(int) * (2 * (size_t)e->grid_tiles + 1),
                          hipHostMallocDefault) == hipSuccess &&
            hipEventCreateWithFlags(&e->ev_upload, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&e->ev_chunk, hipEventDisableTiming) == hipSuccess;
  if (ok && e->method == 1)
    ok = hipHostMalloc((void**)&e->p_sums, sizeof(Summary) * max_sys, hipHostMallocDefault) ==
         hipSuccess;
  if (ok && e->method == 0)   // FP64 and mixed Bi-CGSTAB share the control block layout
    ok = hipHostMalloc((void**)&e->p_ctl, sizeof(BCtl) * max_sys, hipHostMallocDefault) ==
         hipSuccess;
  if (!ok) {
    engine_destroy(e);
    return -5;
  }
  *out = e;
  return 0;
}

void engine_destroy(Engine* e) {
  if (!e) return;
  if (e->s) (void)hipStreamSynchronize(e->s);
  for (auto& kv : e->graphs) (void)hipGraphExecDestroy(kv.second);
  if (e->ev_upload) (void)hipEventDestroy(e->ev_upload);
  if (e->ev_chunk) (void)hipEventDestroy(e->ev_chunk);
  if (e->p_sys) (void)hipHostFree(e->p_sys);
  if (e->p_tiles) (void)hipHostFree(e->p_tiles);
  if (e->p_ctl) (void)hipHostFree(e->p_ctl);
  if (e->p_sums) (void)hipHostFree(e->p_sums);
  delete e;
}

// The pinned staging buffers may be rewritten only after the previous upload has run.
static int wait_upload(Engine& e) {
  if (e.upload_pending) {
    if (hipEventSynchronize(e.ev_upload) != hipSuccess) return -5;
    e.upload_pending = false;
  }
  return 0;
}

int engine_submit(Engine* e, const Mat& A, const double* b, double* x, const SolveParams& prm,
                  int64_t tag, const GsStage* gs) {
  int slot = -1;
  for (int i = 0; i < e->max_sys; ++i)
    if (!e->active[i]) {
      slot = i;
      break;
    }
  if (slot < 0) return 1;   // no free slot
  if (e->mixed && (!gs || !gs->mat32)) return -1;
  const int need = (A.n + BS - 1) / BS;
  const int held = (need + e->rv - 1) / e->rv * e->rv;   // whole units
  int start = 0;
  if (!alloc_tiles(*e, held, start)) return 1;   // no room
  SysDesc d{};
  d.n = A.n;
  d.kind = A.kind;
  d.nx = A.nx;
  d.ny = A.ny;
  d.nz = A.nz;
  d.tile_off = start;
  d.ntiles = need;
  d.unit_off = start / e->rv;
  d.nunits = held / e->rv;
  d.row_off = (int64_t)start * BS;
  d.rp = A.csr.rp;
  d.ci = A.csr.ci;
  d.val = A.csr.val;
  d.coef = A.coef;
  d.b = b;
  d.x = x;
  d.W = prm.weights;
  d.gs_p = 0;
  d.mat32 = nullptr;
  d.ldp32 = 0;
  if (gs && gs->p > 0) {   // the solve reads the GS outputs
    d.gs_p = gs->p;
    d.gs_val = A.kind == MAT_STENCIL ? A.coef : A.csr.val;
    d.gs_b = b;
    if (A.kind == MAT_STENCIL) d.coef = gs->val_out;
    else d.val = gs->val_out;
    d.b = gs->b_out;
    d.W = gs->weight_out;
  }
  if (e->mixed) {
    d.mat32 = gs->mat32;
    d.ldp32 = gs->ldp32;
  }
  const bool prepare = d.gs_p > 0 || d.mat32 != nullptr;
  e->h_sys[slot] = d;
  e->tags[slot] = tag;
  e->active[slot] = 1;
  for (int t = 0; t < held; ++t) e->tile_sys[start + t] = slot;
  e->dirty = true;
  int* bad = nullptr;
  if (e->method == 1) {
    Ctl* c = e->gargs.ctl + slot;
    bad = &c->bad;
    if (launch_gmres_init(c, prm.maxit, e->m, prm.tol, prm.eps_b, d.W ? 1 : 0, prepare ? 1 : 0,
                          e->s) != hipSuccess)
      return -5;
  } else {
    BCtl* c = e->args.ctl + slot;
    bad = &c->bad;
    hipLaunchKernelGGL(k_batch_init, dim3(1), dim3(64), 0, e->s, c, prm.maxit, prm.tol,
                       prm.eps_b, d.W ? 1 : 0, prepare ? 1 : 0);
  }
  if (A.kind == MAT_CSR) {
    int64_t blocks = ((int64_t)A.csr.nnz + A.n + BS) / BS;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_batch_validate, dim3((unsigned)blocks), dim3(BS), 0, e->s, A.csr.rp,
                       A.csr.ci, A.n, A.csr.nnz, bad);
  }
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

static int upload(Engine& e) {
  if (!e.dirty) return 0;
  if (wait_upload(e)) return -5;
  for (int i = 0; i < e.max_sys; ++i) {
    e.p_sys[i] = e.h_sys[i];
    if (!e.active[i]) e.p_sys[i].ntiles = 0;
  }
  int n = 0;
  for (int t = 0; t < e.grid_tiles; t += e.rv) {
    if (e.tile_sys[t] < 0) continue;
    e.p_tiles[n] = t / e.rv;
    e.p_tiles[e.max_units + n] = e.tile_sys[t];
    ++n;
  }
  e.p_tiles[2 * (size_t)e.max_units] = n;
  e.n_listed = n;
  if (hipMemcpyAsync(e.d_sys, e.p_sys, sizeof(SysDesc) * e.max_sys,
                     hipMemcpyHostToDevice, e.s) != hipSuccess ||
      hipMemcpyAsync(e.d_list, e.p_tiles,
                     sizeof(int) * (2 * (size_t)e.max_units + 1), hipMemcpyHostToDevice,
                     e.s) != hipSuccess ||
      hipEventRecord(e.ev_upload, e.s) != hipSuccess)
    return -5;
  e.upload_pending = true;
  e.dirty = false;
  return 0;
}

// Launch of a streaming kernel of class kc; in a sampled chunk (probed == kc) it carries a pair
// of timing events and is followed by the launch that records its algorithmic bytes.
template <class F>
static void launch_stream(Engine& e, F kernel, int kc, int probed, dim3 grid, const BArgsB& a) {
  const int slot = probed == kc ? probe_slot_all(kc) : -1;
  launch_probed(kernel, grid, e.s, slot, a);
  if (slot >= 0)
    hipLaunchKernelGGL(k_batch_probe_bytes, dim3(1), dim3(BS), 0, e.s, a, e.max_sys, kc, slot,
                       e.d_probe);
}

static void enqueue_chunk(Engine& e, int k, int64_t first_iter, int grid, int probed = 0) {
  if (e.method == 1) {
    (void)launch_gmres_chunk(e.gargs, e.m, grid, e.max_sys, e.column, e.s);
    return;
  }
  if (e.mixed) {
    (void)launch_bicg_mixed_chunk(e.margs, k, first_iter, grid, e.max_sys, e.s);
    return;
  }
  const dim3 gt(grid), gs(e.max_sys), block(BS);
  BArgsB a = e.args;
  hipLaunchKernelGGL(k_batch_gs, gt, block, 0, e.s, a);
  hipLaunchKernelGGL(k_batch_fin_gs, gs, dim3(64), 0, e.s, a);
  hipLaunchKernelGGL(k_batch_residual, gt, block, 0, e.s, a);
  hipLaunchKernelGGL(k_batch_fin_residual, gs, block, 0, e.s, a);
  for (int it = 0; it < k; ++it) {
    a.par = (int)((first_iter + it) & 1);
    if (e.rv == 2) launch_stream(e, k_batch_p<2>, KC_BATCH_P, probed, gt, a);
    else launch_stream(e, k_batch_p<1>, KC_BATCH_P, probed, gt, a);
    hipLaunchKernelGGL(k_batch_fin_p, gs, block, 0, e.s, a);
    if (e.rv == 2) launch_stream(e, k_batch_s<2>, KC_BATCH_S, probed, gt, a);
    else launch_stream(e, k_batch_s<1>, KC_BATCH_S, probed, gt, a);
    hipLaunchKernelGGL(k_batch_fin_s, gs, block, 0, e.s, a);
    launch_stream(e, k_batch_u, KC_BATCH_U, probed, gt, a);
    hipLaunchKernelGGL(k_batch_fin_u, gs, block, 0, e.s, a);
  }
}

int engine_run(Engine* e, int chunks) {
  if (upload(*e)) return -5;
  const int k = e->check_every;
  const int grid = stream_grid(e->n_listed);
  hipGraphExec_t exec = nullptr;
  if (e->use_graph) {
    // Every Bi-CGSTAB chunk starts at an even iteration (k is even) and every GMRES chunk at
    // the start of a cycle, so one captured chunk per grid size serves all; the chunk reads
    // the unit list and control blocks from device memory.
    auto it = e->graphs.find(grid);
    if (it != e->graphs.end()) {
      exec = it->second;
    } else {
      hipGraph_t g = nullptr;
      if (hipStreamBeginCapture(e->s, hipStreamCaptureModeThreadLocal) != hipSuccess) return -5;
      enqueue_chunk(*e, k, 0, grid);
      if (hipStreamEndCapture(e->s, &g) != hipSuccess) return -5;
      const hipError_t r = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (r != hipSuccess) return -5;
      e->graphs[grid] = exec;
    }
  }
  // measurement: while a batch kernel class is probed, every probe_every-th chunk is enqueued
  // without its graph, with that class's launches timed
  int probe_cls = 0, every = 0;
  if (e->method == 0 && !e->mixed) {
    for (int kc : {(int)KC_BATCH_P, (int)KC_BATCH_S, (int)KC_BATCH_U})
      if ((every = probe_every(kc)) > 0) {
        probe_cls = kc;
        break;
      }
  }
  for (int c = 0; c < chunks; ++c) {
    const bool sampled = probe_cls && (e->probe_chunks++ % every) == 0;
    if (sampled) {
      if (!e->probe_pending) probe_solve_begin();
      e->probe_pending = true;
      enqueue_chunk(*e, k, e->launched, grid, probe_cls);
    } else if (exec) {
      if (hipGraphLaunch(exec, e->s) != hipSuccess) return -5;
    } else {
      enqueue_chunk(*e, k, e->launched, grid);
    }
    e->launched += k;
  }
  if (hipGetLastError() != hipSuccess) return -5;
  const hipError_t cp =
      e->method == 1
          ? hipMemcpyAsync(e->p_sums, e->gargs.sums, sizeof(Summary) * e->max_sys,
                           hipMemcpyDeviceToHost, e->s)
          : hipMemcpyAsync(e->p_ctl, e->args.ctl, sizeof(BCtl) * e->max_sys,
                           hipMemcpyDeviceToHost, e->s);
  if (cp != hipSuccess || hipEventRecord(e->ev_chunk, e->s) != hipSuccess) return -5;
  e->chunk_pending = true;
  return 0;
}

// Waits for the last enqueued chunk (if wait, or if it has already finished) and retires the
// systems that are done: fills out[] (up to max_out), frees their rows and slots.
int engine_poll(Engine* e, bool wait, EngineDone* out, int max_out, int* n_out) {
  *n_out = 0;
  if (!e->chunk_pending) return 0;
  if (!wait) {
    const hipError_t q = hipEventQuery(e->ev_chunk);
    if (q == hipErrorNotReady) return 0;
    if (q != hipSuccess) return -5;
  } else if (hipEventSynchronize(e->ev_chunk) != hipSuccess) {
    return -5;
  }
  e->chunk_pending = false;
  if (e->probe_pending) {   // the sampled chunk's timed launches and bytes are complete
    probe_collect(e->d_probe, e->s);
    e->probe_pending = false;
  }
  int n = 0;
  for (int i = 0; i < e->max_sys && n < max_out; ++i) {
    if (!e->active[i] || status_of(*e, i).state != ST_DONE) continue;
    out[n].tag = e->tags[i];
    out[n].sum = status_of(*e, i);
    ++n;
    e->active[i] = 0;
    const SysDesc& d = e->h_sys[i];
    const int held = d.nunits * e->rv;
    for (int t = 0; t < held; ++t) e->tile_sys[d.tile_off + t] = -1;
    free_tiles_range(*e, d.tile_off, held);
    e->dirty = true;
  }
  *n_out = n;
  return 0;
}

void engine_usage(const Engine* e, int* active, int64_t* free_rows, int64_t* largest_free_rows) {
  int a = 0;
  for (int i = 0; i < e->max_sys; ++i) a += e->active[i] ? 1 : 0;
  int64_t f = 0, big = 0;
  for (const auto& kv : e->free_tiles) {
    f += kv.second;
    if (kv.second > big) big = kv.second;
  }
  *active = a;
  *free_rows = f * BS;
  *largest_free_rows = big * BS;
}

}  // namespace gsk
