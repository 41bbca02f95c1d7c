// The batch engine's FP64 Bi-CGSTAB workgroup bodies (batch.hip), shared with the
// mixed-precision engine (batch_mixed.hip), whose systems continue in FP64 when float-storage
// refinement stops paying: the same operations in the same order, so a system's FP64 steps
// round identically in either engine.
#pragma once

#include "batch.hpp"

namespace gsk {

struct BArgsB {
  const SysDesc* sys;
  const int* act;        // [2][max_units]: units of one class's systems, then their slots
  const int* n_act;      // number of entries in act
  BCtl* ctl;             // [max_systems]
  double* partials;      // [4][max_tiles]
  int max_tiles;
  int max_units;         // list capacity (its second half starts there)
  int rv;                // tiles per list unit (1 or 2)
  int split;             // per-tile launches: rv workgroups per unit, one tile each
  double* r;
  double* rh;
  double* p[2];
  double* v[2];
  double* t;
  int par;               // buffer parity of this iteration
};

// Calls body(tile, slot) for the tile of this workgroup. Logical block k takes list entry k,
// or with `split` tile k % rv of entry k / rv; consecutive entries, adjacent rows of one
// system, go to one XCD. Without split a unit of two tiles is taken by one workgroup, its
// tiles in turn (the workgroup's LDS is reused between them). Workgroups past the end of the
// list (the launch grid is the list length rounded up) return at once.
template <class Body>
__device__ inline void for_active_tiles(const BArgsB& a, Body body) {
  const int k = logical_block();
  if (a.split) {
    const int e = k / a.rv, q = k - e * a.rv;
    if (e >= *a.n_act) return;
    const int unit = a.act[e], s = a.act[a.max_units + e];
    const int lt = (unit - a.sys[s].unit_off) * a.rv + q;
    if (lt < a.sys[s].ntiles) body(a.sys[s].tile_off + lt, s);
    return;
  }
  if (k >= *a.n_act) return;
  const int unit = a.act[k], s = a.act[a.max_units + k];
  if (a.rv == 1) {
    body(unit, s);
    return;
  }
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

// ---------------------------------------------------------------------------------------
// FP64 bodies. The caller has checked the system's state; each body does one list entry.
// ---------------------------------------------------------------------------------------

// R: r = b - A x over one tile (system-local tile index tile - tile_off); r and r^ are stored
// unless st is ST_FINAL; partials ||r||^2, ||W r||^2.
__device__ inline void bicg64_residual_tile(const BArgsB& a, int tile, int s, int st,
                                            TileLds& L, double* red) {
  const SysDesc d = a.sys[s];
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
}

// P over one unit of two tiles: p = r + beta (p - omega v) (p = r on the first iteration of a
// run), v = A p; partials (r^, v), ||v||^2 per tile.
__device__ inline void bicg64_p_unit2(const BArgsB& a, int unit, int s, UnitLds& U,
                                      double* red) {
  TileLds& L = U.csr;
  const SysDesc d = a.sys[s];
  const BCtl* c = a.ctl + s;
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
}

// S over one unit of two tiles: t = A s with s = r - alpha v; partials (t, s), (t, t), ||s||^2,
// ||W s||^2 per tile.
__device__ inline void bicg64_s_unit2(const BArgsB& a, int unit, int s, UnitLds& U,
                                      double* red) {
  TileLds& L = U.csr;
  const SysDesc d = a.sys[s];
  const BCtl* c = a.ctl + s;
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
}

// U over one tile: x += alpha p + omega s, r = s - omega t; partials (r^, r), ||r||^2, ||W r||^2.
// After a half-step exit (st == ST_HALF) only x += alpha p.
__device__ inline void bicg64_u_tile(const BArgsB& a, int tile, int s, int st, double* red) {
  const SysDesc d = a.sys[s];
  const BCtl* c = a.ctl + s;
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
}

}  // namespace gsk
