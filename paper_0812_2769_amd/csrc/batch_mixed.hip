// Mixed-precision Bi-CGSTAB in the batch engine: iterative refinement whose corrections are
// Bi-CGSTAB runs with FP32 storage (not in the paper, which solves in FP64 throughout; the
// oracle's orc_bicgstab_ir is the definition followed here).
//
//   1. r = b - A x in FP64 with the FP64 scaled matrix; rt = ||W r|| / ||W r0||; the solve
//      stops when rt < tol.
//   2. A run of Bi-CGSTAB restarts from r: the stored residual r~ and the shadow residual r^
//      are r rounded to FP32. The matrix (an FP32 copy), r~, r^, p, v and t are stored as
//      FP32; every product, dot product and update is computed in FP64 from the stored values
//      and rounded to FP32 when it is stored. s = r~ - alpha v is not stored and stays FP64;
//      x stays FP64.
//   3. The run ends (back to 1) when its estimate ||W s|| / ||W r0|| (half step) or
//      ||W r~|| / ||W r0|| drops below max(tol, delta rt), and also when ||W r~|| / ||W r0||
//      exceeds rt / delta or is not finite (the float recurrences have diverged; they can,
//      to overflow, on the jump problems), or after run_cap iterations.
//   A refinement step that does not halve rt counts as a failure. Breakdown tests as in FP64
//   Bi-CGSTAB, on the stored vectors.
//   4. FP64 continuation (orc_bicgstab_ir with fallback, the definition followed here): a run
//      that leaves rt above the value it started from is undone (x := its value at the run's
//      start, saved by the run's first U launch) and the solve continues as FP64 Bi-CGSTAB;
//      so does a solve after three failures in a row, or after a float-storage breakdown
//      (undone first if it left rt higher). The continuation is the FP64 engine's iteration
//      (the bodies of bicg_batch.hpp on FP64 vectors of the engine's row space), from r = b - A x
//      with the same reference norm, iteration count and cap; the hand-over counts as a
//      restart and its iteration count is reported (Summary::fp64_from).
//
// Workgroups take units of two 256-row tiles (FP32 loads carry half the bytes, so a thread
// keeps two rows' loads in flight); partial sums stay per tile, so each system's finalize
// reduces its tiles in order. Float storage costs Bi-CGSTAB iterations on the paper's jump
// problems (each restart discards the Krylov space); this form exists to measure that on the
// device beside the FP64 engine.
#include "bicg_batch.hpp"

namespace gsk {

template <class Body>
__device__ inline void on_unit(const MArgs& a, Body body) {
  const int k = logical_block();
  if (k < *a.n_act) body(a.act[k], a.act[a.max_units + k]);
}

// p = fl(r~ + beta (p - omega v)), or r~ on the first iteration of a run.
struct GatherPM {
  const float* __restrict__ r;
  const float* __restrict__ p;
  const float* __restrict__ v;
  double beta, omega;
  int first;
  struct Raw {
    float r, p, v;
  };
  __device__ Raw load(int col) const { return Raw{r[col], p[col], v[col]}; }
  __device__ double value(const Raw& a) const {
    if (first) return (double)a.r;
    return (double)(float)fma(beta, fma(-omega, (double)a.v, (double)a.p), (double)a.r);
  }
  __device__ double operator()(int col) const { return value(load(col)); }
};

// s = r~ - alpha v (FP64, not stored).
struct GatherSM {
  const float* __restrict__ r;
  const float* __restrict__ v;
  double alpha;
  struct Raw {
    float r, v;
  };
  __device__ Raw load(int col) const { return Raw{r[col], v[col]}; }
  __device__ double value(const Raw& a) const { return fma(-alpha, (double)a.v, (double)a.r); }
  __device__ double operator()(int col) const { return value(load(col)); }
};

// The FP32 product over the two tiles of a unit: y[k] for rows row0[k] .. row0[k] + nr[k].
// Stencil: both tiles' operands are loaded before either sum, and own[k] returns the operands
// of the thread's own row in tile k, which the gather loaded already (own_ok); CSR: one tile
// at a time, and the caller loads the row's operands itself.
template <class G>
__device__ inline void unit_product(const SysDesc& d, const int (&row0)[2], const int (&nr)[2],
                                    const G& g, TileLds& L, double (&y)[2],
                                    typename G::Raw (&own)[2], bool& own_ok) {
  own_ok = false;
  if (d.kind == MAT_STENCIL) {
    const StencilOpT<float> op{d.mat32, d.n, d.nx, d.ny, d.nz, d.ldp32};
    typename StencilOpT<float>::template Pre<G> pre[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) pre[k] = op.load(row0[k], nr[k], g);
    EmptyLds e;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      own[k] = pre[k].centre();
      y[k] = op.finish(pre[k], row0[k], nr[k], g, e);
    }
    own_ok = true;
  } else {
    const CsrOpT<float> op{d.rp, d.ci, d.mat32};
    for (int k = 0; k < 2; ++k) {
      if (k) __syncthreads();
      y[k] = nr[k] > 0 ? op.tile(row0[k], nr[k], g, L) : 0.0;
    }
  }
}

// The engine's FP64 vectors as the FP64 bodies take them (units of two tiles).
__device__ inline BArgsB fp64_view(const MArgs& a) {
  BArgsB b;
  b.sys = a.sys;
  b.act = a.act;
  b.n_act = a.n_act;
  b.ctl = a.ctl;
  b.partials = a.partials;
  b.max_tiles = a.pstride;
  b.max_units = a.max_units;
  b.rv = 2;
  b.split = 0;
  b.r = a.r64;
  b.rh = a.rh64;
  b.p[0] = a.p64[0];
  b.p[1] = a.p64[1];
  b.v[0] = a.v64[0];
  b.v[1] = a.v64[1];
  b.t = a.t64;
  b.par = a.par;
  return b;
}

__device__ inline void unit_rows(const SysDesc& d, int unit, int& lt0, int (&row0)[2],
                                 int (&nr)[2]) {
  lt0 = (unit - d.unit_off) * 2;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    row0[k] = (lt0 + k) * BS;
    nr[k] = max(0, min(BS, d.n - row0[k]));
  }
}

__global__ __launch_bounds__(BS) void k_bm_prepare(MArgs a) {
  __shared__ GsLds L;
  on_unit(a, [&](int unit, int s) {
    const SysDesc d = a.sys[s];
    BCtl* c = a.ctl + s;
    if (c->sum.state == ST_ROLLBACK) {   // undo the last float run
      const int lt0 = (unit - d.unit_off) * 2;
      for (int k = 0; k < 2; ++k) {
        const int row = (lt0 + k) * BS + (int)threadIdx.x;
        if (row < d.n) d.x[row] = a.xprev[d.row_off + row];
      }
      return;
    }
    if (c->sum.state != ST_SCALE || (c->bad & BAD_CSR)) return;
    const int lt0 = (unit - d.unit_off) * 2;
    for (int k = 0; k < 2; ++k) {
      if (lt0 + k >= d.ntiles) break;
      prepare_tile(d, lt0 + k, L, &c->bad);
      __syncthreads();
    }
  });
}

__global__ __launch_bounds__(64) void k_bm_fin_prepare(MArgs a) {
  const int s = blockIdx.x;
  if (threadIdx.x != 0 || a.sys[s].ntiles == 0) return;
  BCtl* c = a.ctl + s;
  if (c->sum.state == ST_SCALE) c->sum.state = ST_INIT;
  else if (c->sum.state == ST_ROLLBACK) c->sum.state = ST_FP64START;
}

// R: r = b - A x (FP64 matrix), r~ = r^ = fl(r) when a run starts; partials ||r||^2,
// ||W r||^2, ||r~||^2 per tile.
__global__ __launch_bounds__(BS) void k_bm_residual(MArgs a) {
  __shared__ TileLds L;
  __shared__ double red[NC_MAX * WAVES];
  on_unit(a, [&](int unit, int s) {
    const SysDesc d = a.sys[s];
    BCtl* c = a.ctl + s;
    const int st = c->sum.state;
    const int lt0 = (unit - d.unit_off) * 2;
    if (c->fp64) {   // FP64 continuation: the FP64 engine's residual
      if (st != ST_FP64START && st != ST_VERIFY && st != ST_FINAL) return;
      const BArgsB b = fp64_view(a);
      for (int k = 0; k < 2 && lt0 + k < d.ntiles; ++k) {
        if (k) __syncthreads();
        bicg64_residual_tile(b, d.tile_off + lt0 + k, s, st, L, red);
      }
      return;
    }
    if (st != ST_INIT && st != ST_VERIFY && st != ST_FINAL) return;
    if (c->bad) return;
    const int t = threadIdx.x;
    for (int k = 0; k < 2; ++k) {
      const int row0 = (lt0 + k) * BS;
      const int nrows = min(BS, d.n - row0);
      if (nrows <= 0) break;
      if (k) __syncthreads();
      double y;
      if (d.kind == MAT_STENCIL) {
        EmptyLds e;
        y = StencilOp{d.coef, d.n, d.nx, d.ny, d.nz, (size_t)d.n}.tile(row0, nrows, GatherX{d.x}, e);
      } else {
        y = CsrOp{d.rp, d.ci, d.val}.tile(row0, nrows, GatherX{d.x}, L);
      }
      double acc[3] = {0.0, 0.0, 0.0};
      if (t < nrows) {
        const int row = row0 + t;
        const double r = d.b[row] - y;
        const float rs = (float)r;
        if (st != ST_FINAL) {
          a.r[d.row_off + row] = rs;
          a.rh[d.row_off + row] = rs;
        }
        acc[0] = r * r;
        if (d.W) {
          const double wr = d.W[row] * r;
          acc[1] = wr * wr;
        }
        acc[2] = (double)rs * (double)rs;
      }
      block_partials<3>(acc, 3, a.partials, a.pstride, d.tile_off + lt0 + k, red);
    }
  });
}

// FR: convergence test on the FP64 residual, refinement bookkeeping, start of a run.
// Hand-over to the FP64 continuation (thread 0 of a finalize workgroup): undo the last run
// first if it left the true residual rt above the value it started from.
__device__ inline void hand_over(BCtl* c, double rt) {
  c->fp64 = 1;
  c->sum.fp64_from = c->sum.iters;
  c->sum.restarts += 1;
  c->sum.fails = 0;
  c->sum.status = S_MAXIT;
  c->sum.brk = BRK_NONE;
  c->target = c->tol;
  c->sum.state = rt <= c->last_rt ? ST_FP64START : ST_ROLLBACK;
}

// FR: convergence test on the FP64 residual, refinement bookkeeping, start of a run; for a
// system in FP64 the FP64 engine's rule (verification, restart, three failures: STAGNATED).
__global__ __launch_bounds__(BS) void k_bm_fin_residual(MArgs a) {
  const int s = blockIdx.x;
  const SysDesc d = a.sys[s];
  if (d.ntiles == 0) return;
  BCtl* c = a.ctl + s;
  const int st = c->sum.state;
  const bool f64 = c->fp64 != 0;
  if (st != ST_INIT && st != ST_VERIFY && st != ST_FINAL && !(f64 && st == ST_FP64START))
    return;
  if (c->bad) {
    if (threadIdx.x == 0) {
      c->sum.state = ST_DONE;
      c->sum.status = bad_status(c->bad);
    }
    return;
  }
  __shared__ double out[8];
  small_sums_strided<3>(a.partials + d.tile_off, d.ntiles, a.pstride, out);
  if (threadIdx.x != 0) return;
  const double nr = sqrt(out[0]);
  const double nwr = d.W ? sqrt(out[1]) : nr;
  if (f64) {
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
    if (st == ST_VERIFY) {
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
    return;
  }
  const double ns = sqrt(out[2]);
  double rt = 1.0;
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
    rt = nwr / c->ref;
    c->sum.relres_true = rt;
    if (st == ST_FINAL) {   // a float-storage run broke down
      hand_over(c, rt);
      return;
    }
    if (rt < c->tol) {
      c->sum.status = S_CONVERGED;
      c->sum.state = ST_DONE;
      return;
    }
    if (!(rt <= c->last_rt)) {   // the run made x worse
      hand_over(c, rt);
      return;
    }
    if (c->sum.iters >= c->maxit) {
      c->sum.status = S_MAXIT;
      c->sum.state = ST_DONE;
      return;
    }
    if (!(rt < 0.5 * c->last_rt)) {
      c->sum.fails += 1;
      if (c->sum.fails >= 3) {
        hand_over(c, rt);
        return;
      }
    } else {
      c->sum.fails = 0;
    }
    c->sum.restarts += 1;
  }
  c->last_rt = rt;
  c->target = a.delta * rt > c->tol ? a.delta * rt : c->tol;
  c->run_start = c->sum.iters;
  c->rh_norm = ns;
  c->rho = out[2];
  c->sum.half = 0;
  if (fabs(c->rho) <= c->eps_b * ns * ns) {
    hand_over(c, rt);   // float-storage breakdown at the start of a run (x unchanged)
    return;
  }
  c->first = 1;
  c->sum.state = ST_RUNNING;
}

// P: p (stored FP32), v = fl(A p); partials (r^, v), ||v||^2.
__global__ __launch_bounds__(BS) void k_bm_p(MArgs a) {
  __shared__ UnitLds U;
  TileLds& L = U.csr;
  __shared__ double red[NC_MAX * WAVES];
  on_unit(a, [&](int unit, int s) {
    const SysDesc d = a.sys[s];
    BCtl* c = a.ctl + s;
    if (c->sum.state != ST_RUNNING) return;
    if (c->fp64) {
      bicg64_p_unit2(fp64_view(a), unit, s, U, red);
      return;
    }
    const int q = a.par;
    const int64_t o = d.row_off;
    const GatherPM G{a.r + o, a.p[q] + o, a.v[q] + o, c->beta, c->omega, c->first};
    int lt0, row0[2], nr[2];
    unit_rows(d, unit, lt0, row0, nr);
    double y[2];
    typename GatherPM::Raw own[2];
    bool own_ok;
    unit_product(d, row0, nr, G, L, y, own, own_ok);
    const int t = threadIdx.x;
    for (int k = 0; k < 2; ++k) {
      if (nr[k] <= 0) break;
      if (k) __syncthreads();
      double acc[2] = {0.0, 0.0};
      if (t < nr[k]) {
        const int row = row0[k] + t;
        a.p[q ^ 1][o + row] = (float)(own_ok ? G.value(own[k]) : G(row));
        const float vs = (float)y[k];
        a.v[q ^ 1][o + row] = vs;
        acc[0] = (double)a.rh[o + row] * (double)vs;
        acc[1] = (double)vs * (double)vs;
      }
      block_partials<2>(acc, 2, a.partials, a.pstride, d.tile_off + lt0 + k, red);
    }
  });
}

__global__ __launch_bounds__(BS) void k_bm_fin_p(MArgs a) {
  const int s = blockIdx.x;
  const SysDesc d = a.sys[s];
  if (d.ntiles == 0) return;
  BCtl* c = a.ctl + s;
  if (c->sum.state != ST_RUNNING) return;
  __shared__ double out[8];
  small_sums_strided<2>(a.partials + d.tile_off, d.ntiles, a.pstride, out);
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

// S: t = fl(A s) with s = r~ - alpha v; partials (t, s), (t, t), ||s||^2, ||W s||^2.
__global__ __launch_bounds__(BS) void k_bm_s(MArgs a) {
  __shared__ UnitLds U;
  TileLds& L = U.csr;
  __shared__ double red[NC_MAX * WAVES];
  on_unit(a, [&](int unit, int s) {
    const SysDesc d = a.sys[s];
    BCtl* c = a.ctl + s;
    if (c->sum.state != ST_RUNNING) return;
    if (c->fp64) {
      bicg64_s_unit2(fp64_view(a), unit, s, U, red);
      return;
    }
    const int64_t o = d.row_off;
    const GatherSM G{a.r + o, a.v[a.par ^ 1] + o, c->alpha};
    int lt0, row0[2], nr[2];
    unit_rows(d, unit, lt0, row0, nr);
    double y[2];
    typename GatherSM::Raw own[2];
    bool own_ok;
    unit_product(d, row0, nr, G, L, y, own, own_ok);
    const int t = threadIdx.x;
    for (int k = 0; k < 2; ++k) {
      if (nr[k] <= 0) break;
      if (k) __syncthreads();
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      if (t < nr[k]) {
        const int row = row0[k] + t;
        const double sv = own_ok ? G.value(own[k]) : G(row);
        const float ts = (float)y[k];
        a.t[o + row] = ts;
        acc[0] = (double)ts * sv;
        acc[1] = (double)ts * (double)ts;
        acc[2] = sv * sv;
        if (d.W) {
          const double ws = d.W[row] * sv;
          acc[3] = ws * ws;
        }
      }
      block_partials<4>(acc, 4, a.partials, a.pstride, d.tile_off + lt0 + k, red);
    }
  });
}

__global__ __launch_bounds__(BS) void k_bm_fin_s(MArgs a) {
  const int s = blockIdx.x;
  const SysDesc d = a.sys[s];
  if (d.ntiles == 0) return;
  BCtl* c = a.ctl + s;
  if (c->sum.state != ST_RUNNING) return;
  __shared__ double out[8];
  small_sums_strided<4>(a.partials + d.tile_off, d.ntiles, a.pstride, out);
  if (threadIdx.x != 0) return;
  c->sum.iters += 1;
  const double sn = sqrt(out[2]);
  const double est = (d.W ? sqrt(out[3]) : sn) / c->ref;
  c->sum.relres_rec = est;
  if (est < c->target) {
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

// U: x += alpha p + omega s (FP64 x), r~ = fl(s - omega t); partials (r^, r~), ||r~||^2,
// ||W r~||^2. After a half-step exit only x += alpha p. The first U of a run saves x as it was
// at the run's start (for the undo of a run that diverged).
__global__ __launch_bounds__(BS) void k_bm_u(MArgs a) {
  __shared__ double red[NC_MAX * WAVES];
  on_unit(a, [&](int unit, int s) {
    const SysDesc d = a.sys[s];
    BCtl* c = a.ctl + s;
    const int st = c->sum.state;
    if (st != ST_RUNNING && st != ST_HALF) return;
    const int lt0 = (unit - d.unit_off) * 2;
    if (c->fp64) {
      const BArgsB b = fp64_view(a);
      for (int k = 0; k < 2 && lt0 + k < d.ntiles; ++k) {
        if (k) __syncthreads();
        bicg64_u_tile(b, d.tile_off + lt0 + k, s, st, red);
      }
      return;
    }
    const int q = a.par ^ 1;
    const int64_t o = d.row_off;
    const float* p = a.p[q] + o;
    const float* v = a.v[q] + o;
    const double alpha = c->alpha, omega = c->omega;
    const bool first = c->first != 0;
    for (int k = 0; k < 2; ++k) {
      const int r0 = (lt0 + k) * BS;
      if (r0 >= d.n) break;
      const int row = r0 + threadIdx.x;
      const bool mine = row < d.n;
      if (st == ST_HALF) {
        if (mine) {
          const double xo = d.x[row];
          if (first) a.xprev[o + row] = xo;
          d.x[row] = fma(alpha, (double)p[row], xo);
        }
        continue;
      }
      if (k) __syncthreads();
      double acc[3] = {0.0, 0.0, 0.0};
      if (mine) {
        const double sv = fma(-alpha, (double)v[row], (double)a.r[o + row]);
        const double xo = d.x[row];
        if (first) a.xprev[o + row] = xo;
        d.x[row] = fma(omega, sv, fma(alpha, (double)p[row], xo));
        const float rs = (float)fma(-omega, (double)a.t[o + row], sv);
        a.r[o + row] = rs;
        acc[0] = (double)a.rh[o + row] * (double)rs;
        acc[1] = (double)rs * (double)rs;
        if (d.W) {
          const double wr = d.W[row] * (double)rs;
          acc[2] = wr * wr;
        }
      }
      block_partials<3>(acc, 3, a.partials, a.pstride, d.tile_off + lt0 + k, red);
    }
  });
}

__global__ __launch_bounds__(BS) void k_bm_fin_u(MArgs a) {
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
  small_sums_strided<3>(a.partials + d.tile_off, d.ntiles, a.pstride, out);
  if (threadIdx.x != 0) return;
  const double rn = sqrt(out[1]);
  const double est = (d.W ? sqrt(out[2]) : rn) / c->ref;
  c->sum.relres_rec = est;
  const bool run_end = !c->fp64 && (!(est <= c->last_rt / a.delta) ||
                                     (a.run_cap > 0 && c->sum.iters - c->run_start >= a.run_cap));
  if (est < c->target || c->sum.iters >= c->maxit || run_end) {
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

hipError_t launch_bicg_mixed_chunk(MArgs a, int k, int64_t first_iter, int grid, int max_sys,
                                   hipStream_t s) {
  const dim3 gt(grid), gs(max_sys), block(BS);
  hipLaunchKernelGGL(k_bm_prepare, gt, block, 0, s, a);
  hipLaunchKernelGGL(k_bm_fin_prepare, gs, dim3(64), 0, s, a);
  hipLaunchKernelGGL(k_bm_residual, gt, block, 0, s, a);
  hipLaunchKernelGGL(k_bm_fin_residual, gs, block, 0, s, a);
  for (int it = 0; it < k; ++it) {
    a.par = (int)((first_iter + it) & 1);
    hipLaunchKernelGGL(k_bm_p, gt, block, 0, s, a);
    hipLaunchKernelGGL(k_bm_fin_p, gs, block, 0, s, a);
    hipLaunchKernelGGL(k_bm_s, gt, block, 0, s, a);
    hipLaunchKernelGGL(k_bm_fin_s, gs, block, 0, s, a);
    hipLaunchKernelGGL(k_bm_u, gt, block, 0, s, a);
    hipLaunchKernelGGL(k_bm_fin_u, gs, block, 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace gsk
