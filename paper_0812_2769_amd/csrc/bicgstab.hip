// Bi-CGSTAB (van der Vorst; section 2 of the paper) on the device, shadow residual r^ = r0.
//
// One iteration is three streaming launches, each followed by a finalize launch that sums the
// per-tile partials in a fixed order (one workgroup; for systems of many tiles four one-wave
// workgroups with the same additions, see split_sums); every scalar stays on the device:
//
//   P  p = r + beta (p - omega v)       (p = r on the first iteration after a (re)start)
//      v = A p, with the p entries of neighbouring rows recomputed inside the gather, so p
//      is written once and never re-read for the product;  (r^, v), ||v||
//      FP -> alpha = rho / (r^, v)
//   S  s = r - alpha v (recomputed in the gather, never stored), t = A s;
//      (t, s), (t, t), ||s||, ||W s||   FS -> half-step test, omega = (t, s) / (t, t)
//   U  x += alpha p + omega s, r = s - omega t; (r^, r), ||r||, ||W r||
//      FU -> stop test, rho, beta
//
// p and v are double-buffered because P reads the old p and v of neighbouring rows while it
// writes the new ones. The host gives every enqueued iteration its buffer parity (the
// iteration's enqueue count mod 2): within a run of working iterations the parities
// alternate, and the first iteration after a (re)start reads no old p or v. The step
// launches request all their operands before they read the control block to learn whether
// they have work (a launch without work stores nothing). The residual launch R computes
// r = b - A x for the initial residual and for every verification of a recursive
// convergence claim; a failed verification restarts the recurrence from the true residual.
#include <mutex>
#include <type_traits>

#include "bicg_batch.hpp"   // the LDS-window workgroup bodies shared with the batch engine
#include "gsk_host.hpp"

namespace gsk {

struct BArgs {
  int n;
  int rpb;
  Ctl* ctl;
  double* partials;
  double* r;
  double* rh;
  double* p[2];
  double* v[2];
  double* t;
  double* x;
  const double* b;
  const double* W;
  double mat_bytes;   // algorithmic bytes of one read of A
  int pslot;          // measurement slot of this launch, or -1
  int par;            // buffer parity of this iteration: reads p[par], v[par]
};

__device__ inline void brange(const BArgs& a, int lb, int& begin, int& end) {
  begin = lb * a.rpb;
  end = min(a.n, begin + a.rpb);
  if (begin > a.n) begin = a.n;
}

__global__ __launch_bounds__(64) void k_bicg_init_ctl(Ctl* c, int maxit, double tol, double eps_b,
                                                      int has_w) {
  for (int i = threadIdx.x; i < PROBE_SLOTS; i += 64) c->probe.bytes[i] = 0.0;
  if (threadIdx.x != 0) return;
  c->sum.state = ST_INIT;
  c->sum.status = S_MAXIT;
  c->sum.iters = 0;
  c->sum.restarts = 0;
  c->sum.half = 0;
  c->sum.fails = 0;
  c->sum.steps = 0;
  c->sum.relres_rec = 1.0;
  c->sum.relres_true = 1.0;
  c->sum.brk = BRK_NONE;
  c->sum.fp64_from = 0;
  c->sum.pad0 = 0;
  c->maxit = maxit;
  c->m = 0;
  c->j = c->k = c->claimed = 0;
  c->first = 1;
  c->has_w = has_w;
  c->broke = c->happy = 0;
  c->tol = tol;
  c->eps_b = eps_b;
  c->ref = 0.0;
  c->ratio = 1.0;
  c->rho = c->rho_old = c->alpha = c->omega = c->beta = c->rh_norm = 0.0;
  c->fin_count = 0;
}

// R: r = b - A x, r^ = r (initial residual, verification, or final residual after a
// breakdown); partials ||r||^2, ||W r||^2.
template <class Op>
__global__ __launch_bounds__(BS) void k_bicg_residual(BArgs a, Op op, const int* flags) {
  Ctl* c = a.ctl;
  const int st = c->sum.state;
  if (st != ST_INIT && st != ST_VERIFY && st != ST_FINAL) return;
  if (flags[0]) return;
  mark_work(c, a.pslot, a.mat_bytes + 8.0 * a.n * ((st != ST_FINAL ? 4 : 2) + (a.W ? 1 : 0)));
  __shared__ typename Op::Lds L;
  __shared__ double red[NC_MAX * WAVES];
  const int nb = gridDim.x;
  const int lb = logical_block();
  int rb, re;
  brange(a, lb, rb, re);
  double acc[2] = {0.0, 0.0};
  for (int row0 = rb; row0 < re; row0 += BS) {
    const int nrows = min(BS, re - row0);
    const double y = op.tile(row0, nrows, GatherX{a.x}, L);
    if ((int)threadIdx.x < nrows) {
      const int row = row0 + threadIdx.x;
      const double r = a.b[row] - y;
      if (st != ST_FINAL) {
        a.r[row] = r;
        a.rh[row] = r;
      }
      acc[0] += r * r;
      if (a.W) {
        const double wr = a.W[row] * r;
        acc[1] += wr * wr;
      }
    }
  }
  block_partials<2>(acc, 2, a.partials, nb, lb, red);
}

// FR: reference residual, convergence check of a verification, or (re)start of the recurrence.
__global__ __launch_bounds__(BS) void k_bicg_fin_residual(Ctl* c, const double* partials, int nb,
                                                          int has_w, const int* flags) {
  const int st = c->sum.state;
  if (st != ST_INIT && st != ST_VERIFY && st != ST_FINAL) return;
  if (flags[0]) {
    if (threadIdx.x == 0) {
      c->sum.state = ST_DONE;
      c->sum.status = -1;
    }
    return;
  }
  __shared__ double out[8];
  small_sums<2>(partials, nb, out);
  if (threadIdx.x != 0) return;
  const double nr = sqrt(out[0]);
  const double nwr = has_w ? sqrt(out[1]) : nr;
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
      c->sum.state = ST_DONE;   // status (breakdown) already set
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
  // (re)start the recurrence from r: r^ = r, rho = (r^, r)
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

// p update, shared by the row's own value and the gather of its neighbours (explicit fma so
// both evaluations round identically).
struct GatherP {
  const double* __restrict__ r;
  const double* __restrict__ p;
  const double* __restrict__ v;
  double beta, omega;
  int first;
  struct Raw {
    double r, p, v;
  };
  __device__ Raw load(int col) const { return Raw{r[col], p[col], v[col]}; }
  __device__ double value(const Raw& a) const {
    return first ? a.r : fma(beta, fma(-omega, a.v, a.p), a.r);
  }
  __device__ double operator()(int col) const { return value(load(col)); }
};

struct GatherS {
  const double* __restrict__ r;
  const double* __restrict__ v;
  double alpha;
  struct Raw {
    double r, v;
  };
  __device__ Raw load(int col) const { return Raw{r[col], v[col]}; }
  __device__ double value(const Raw& a) const { return fma(-alpha, a.v, a.r); }
  __device__ double operator()(int col) const { return value(load(col)); }
};

// P: new p, v = A p; partials (r^, v), ||v||^2.
template <class Op>
__global__ __launch_bounds__(BS) void k_bicg_p(BArgs a, Op op) {
  Ctl* c = a.ctl;
  const int state = c->sum.state, first = c->first;
  const double beta = c->beta, omega = c->omega;
  const int q = a.par;
  const GatherP G{a.r, a.p[q], a.v[q], beta, omega, first};
  __shared__ typename Op::Lds L;
  __shared__ double red[NC_MAX * WAVES];
  const int nb = gridDim.x;
  const int lb = logical_block();
  const int row0 = lb * BS;
  const int nrows = max(0, min(BS, a.n - row0));
  const int t = threadIdx.x;
  const bool mine = t < nrows;
  const int row = mine ? row0 + t : 0;
  const double rhv = a.rh[row];
  typename Op::template Pre<GatherP> pre{};
  if (nrows > 0) pre = op.load(row0, nrows, G);
  GatherP::Raw own;
  if constexpr (Op::kRowwise) own = pre.centre();   // a stencil row gathers its own entries
  else own = G.load(row);
  asm volatile("" ::: "memory");   // every load above is issued before anything is combined
  // A CSR product follows indices that are trusted only while the solve runs: test first.
  if constexpr (!Op::kRowwise) {
    if (state != ST_RUNNING) return;
  }
  const double y = nrows > 0 ? op.finish(pre, row0, nrows, G, L) : 0.0;
  const double pn = G.value(own);
  if (state != ST_RUNNING) return;
  mark_work(c, a.pslot, a.mat_bytes + 8.0 * a.n * (first ? 4 : 6));
  double acc[2] = {0.0, 0.0};
  if (mine) {
    a.p[q ^ 1][row] = pn;
    a.v[q ^ 1][row] = y;
    acc[0] = rhv * y;
    acc[1] = y * y;
  }
  block_partials<2>(acc, 2, a.partials, nb, lb, red);
}

// ---------------------------------------------------------------------------------------
// P and S for a stencil matrix through the LDS window of the batch engine's bodies: one
// workgroup per two tiles; the gathered values of the tiles' rows and one x-line on either
// side are formed once into LDS, rows read in 16-byte pairs where n and nx are even. Every
// tile's partials are reduced in the order of the one-tile kernels above, so the results are
// the same bits. The control words are read first and tested after the window is formed (its
// loads are clamped, valid addresses in any state). Partial slots of tiles past the matrix
// (the partial stride nb is the tile grid) are written as zeros, as the one-tile kernels do.
// ---------------------------------------------------------------------------------------
constexpr int kWindowRows = 1 << 20;   // systems from this size on take the window kernels

__device__ inline SysDesc window_sys(const StencilOp& op, const double* W) {
  SysDesc d{};
  d.n = op.n;
  d.kind = MAT_STENCIL;
  d.nx = op.nx;
  d.ny = op.ny;
  d.nz = op.nz;
  d.coef = op.coef;
  d.W = W;
  return d;
}

template <int NC>
__device__ inline void zero_tail_partials(double* partials, int nb, int tiles, int lt0) {
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int tile = lt0 + k;
    if (tile >= tiles && tile < nb && threadIdx.x < NC)
      partials[(size_t)threadIdx.x * nb + tile] = 0.0;
  }
}

__global__ __launch_bounds__(BS) void k_bicg_p_win(BArgs a, StencilOp op, int nb) {
  __shared__ UnitLds U;
  __shared__ double red[NC_MAX * WAVES];
  Ctl* c = a.ctl;
  const int state = c->sum.state, first = c->first;
  const double beta = c->beta, omega = c->omega;
  const int q = a.par;
  const GatherPB G{a.r, a.p[q], a.v[q], beta, omega, first};
  const SysDesc d = window_sys(op, nullptr);
  const int tiles = (a.n + BS - 1) / BS;
  const int lt0 = 2 * logical_block();
  if (lt0 >= tiles) {
    if (state == ST_RUNNING) zero_tail_partials<2>(a.partials, nb, tiles, lt0);
    return;
  }
  const int R0 = lt0 * BS, nu = min(2 * BS, a.n - R0);
  const bool pair = unit_pairs(d, nullptr);
  int row[2];
  bool ok[2];
  double y[2], gv[2];
  unit_window(d, R0, nu, pair, G, U.g, row, ok, y, gv);
  double rh[2];
  if (pair) {
    const double2 r2 = ld2(a.rh + row[0]);
    rh[0] = r2.x;
    rh[1] = r2.y;
  } else {
    rh[0] = a.rh[row[0]];
    rh[1] = a.rh[row[1]];
  }
  if (state != ST_RUNNING) return;
  mark_work(c, a.pslot, a.mat_bytes + 8.0 * a.n * (first ? 4 : 6));
  double acc[2][2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    acc[h][0] = ok[h] ? rh[h] * y[h] : 0.0;
    acc[h][1] = ok[h] ? y[h] * y[h] : 0.0;
  }
  if (pair) {
    if (ok[0]) {
      *reinterpret_cast<double2*>(a.p[q ^ 1] + row[0]) = double2{gv[0], gv[1]};
      *reinterpret_cast<double2*>(a.v[q ^ 1] + row[0]) = double2{y[0], y[1]};
    }
  } else {
#pragma unroll
    for (int h = 0; h < 2; ++h)
      if (ok[h]) {
        a.p[q ^ 1][row[h]] = gv[h];
        a.v[q ^ 1][row[h]] = y[h];
      }
  }
  unit_partials<2>(pair, acc, U.acc, min(2, tiles - lt0), a.partials, nb, lt0, red);
  zero_tail_partials<2>(a.partials, nb, tiles, lt0);
}

__global__ __launch_bounds__(BS) void k_bicg_s_win(BArgs a, StencilOp op, int nb) {
  __shared__ UnitLds U;
  __shared__ double red[NC_MAX * WAVES];
  Ctl* c = a.ctl;
  const int state = c->sum.state;
  const GatherSB G{a.r, a.v[a.par ^ 1], c->alpha};   // the v written by P in this iteration
  const SysDesc d = window_sys(op, a.W);
  const int tiles = (a.n + BS - 1) / BS;
  const int lt0 = 2 * logical_block();
  if (lt0 >= tiles) {
    if (state == ST_RUNNING) zero_tail_partials<4>(a.partials, nb, tiles, lt0);
    return;
  }
  const int R0 = lt0 * BS, nu = min(2 * BS, a.n - R0);
  const bool pair = unit_pairs(d, a.W);
  int row[2];
  bool ok[2];
  double y[2], sv[2];
  unit_window(d, R0, nu, pair, G, U.g, row, ok, y, sv);
  double wv[2] = {0.0, 0.0};
  if (a.W) {
    if (pair) {
      const double2 w2 = ld2(a.W + row[0]);
      wv[0] = w2.x;
      wv[1] = w2.y;
    } else {
      wv[0] = a.W[row[0]];
      wv[1] = a.W[row[1]];
    }
  }
  if (state != ST_RUNNING) return;
  mark_work(c, a.pslot, a.mat_bytes + 8.0 * a.n * (a.W ? 4 : 3));
  double acc[2][4];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    acc[h][0] = ok[h] ? y[h] * sv[h] : 0.0;
    acc[h][1] = ok[h] ? y[h] * y[h] : 0.0;
    acc[h][2] = ok[h] ? sv[h] * sv[h] : 0.0;
    const double ws = wv[h] * sv[h];
    acc[h][3] = ok[h] && a.W ? ws * ws : 0.0;
  }
  if (pair) {
    if (ok[0]) *reinterpret_cast<double2*>(a.t + row[0]) = double2{y[0], y[1]};
  } else {
#pragma unroll
    for (int h = 0; h < 2; ++h)
      if (ok[h]) a.t[row[h]] = y[h];
  }
  unit_partials<4>(pair, acc, U.acc, min(2, tiles - lt0), a.partials, nb, lt0, red);
  zero_tail_partials<4>(a.partials, nb, tiles, lt0);
}

// FP: alpha = rho / (r^, v), or breakdown. (The finalize launches read their control words
// together with the partials, one memory round trip, and only the stores depend on them.)
template <bool BIG>
__global__ __launch_bounds__(BS) void k_bicg_fin_p(Ctl* c, const double* partials, int nb) {
  const int state = c->sum.state;
  const double eps_b = c->eps_b, rh_norm = c->rh_norm, rho = c->rho;
  __shared__ double out[8];
  if constexpr (BIG) {
    if (!split_sums<2, sum_batch<2>()>(c, partials, nb, out)) return;
  } else {
    small_sums<2, SUM_BATCH>(partials, nb, out);
  }
  if (state != ST_RUNNING || threadIdx.x != 0) return;
  const double sigma = out[0];
  const double vn = sqrt(out[1]);
  if (fabs(sigma) <= eps_b * rh_norm * vn) {
    c->sum.status = S_BREAKDOWN;
    c->sum.brk = BRK_SIGMA;
    c->sum.state = ST_FINAL;
    return;
  }
  c->alpha = rho / sigma;
}

// S: t = A s with s = r - alpha v; partials (t,s), (t,t), ||s||^2, ||W s||^2.
template <class Op>
__global__ __launch_bounds__(BS) void k_bicg_s(BArgs a, Op op) {
  Ctl* c = a.ctl;
  const int state = c->sum.state;
  const double alpha = c->alpha;
  const GatherS G{a.r, a.v[a.par ^ 1], alpha};   // the v written by P in this iteration
  __shared__ typename Op::Lds L;
  __shared__ double red[NC_MAX * WAVES];
  const int nb = gridDim.x;
  const int lb = logical_block();
  const int row0 = lb * BS;
  const int nrows = max(0, min(BS, a.n - row0));
  const int t = threadIdx.x;
  const bool mine = t < nrows;
  const int row = mine ? row0 + t : 0;
  const double wv = a.W ? a.W[row] : 0.0;
  typename Op::template Pre<GatherS> pre{};
  if (nrows > 0) pre = op.load(row0, nrows, G);
  GatherS::Raw own;
  if constexpr (Op::kRowwise) own = pre.centre();   // a stencil row gathers its own entries
  else own = G.load(row);
  asm volatile("" ::: "memory");
  if constexpr (!Op::kRowwise) {
    if (state != ST_RUNNING) return;
  }
  const double y = nrows > 0 ? op.finish(pre, row0, nrows, G, L) : 0.0;
  const double sv = G.value(own);
  if (state != ST_RUNNING) return;
  mark_work(c, a.pslot, a.mat_bytes + 8.0 * a.n * (a.W ? 4 : 3));
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (mine) {
    a.t[row] = y;
    acc[0] = y * sv;
    acc[1] = y * y;
    acc[2] = sv * sv;
    if (a.W) {
      const double ws = wv * sv;
      acc[3] = ws * ws;
    }
  }
  block_partials<4>(acc, 4, a.partials, nb, lb, red);
}

// FS: iteration count, half-step test on ||W s||, omega = (t,s)/(t,t), or breakdown.
template <bool BIG>
__global__ __launch_bounds__(BS) void k_bicg_fin_s(Ctl* c, const double* partials, int nb,
                                                   int has_w) {
  const int state = c->sum.state, iters = c->sum.iters;
  const double ref = c->ref, tol = c->tol, eps_b = c->eps_b;
  __shared__ double out[8];
  if constexpr (BIG) {
    if (!split_sums<4, sum_batch<4>()>(c, partials, nb, out)) return;
  } else {
    small_sums<4, SUM_BATCH>(partials, nb, out);
  }
  if (state != ST_RUNNING || threadIdx.x != 0) return;
  c->sum.iters = iters + 1;
  const double sn = sqrt(out[2]);
  const double est = (has_w ? sqrt(out[3]) : sn) / ref;
  c->sum.relres_rec = est;
  if (est < tol) {
    c->sum.half = 1;
    c->sum.state = ST_HALF;
    return;
  }
  const double ts = out[0], tt = out[1];
  if (fabs(ts) <= eps_b * sqrt(tt) * sn) {
    c->sum.status = S_BREAKDOWN;
    c->sum.brk = BRK_OMEGA;
    c->sum.state = ST_FINAL;
    return;
  }
  c->omega = ts / tt;
}

// U: x += alpha p + omega s, r = s - omega t; partials (r^, r), ||r||^2, ||W r||^2.
// After a half-step exit only x += alpha p is done.
__global__ __launch_bounds__(BS) void k_bicg_u(BArgs a) {
  Ctl* c = a.ctl;
  const int st = c->sum.state;
  const double alpha = c->alpha, omega = c->omega;
  const int q = a.par ^ 1;   // p and v written by P in this iteration
  __shared__ double red[NC_MAX * WAVES];
  const int nb = gridDim.x;
  const int lb = logical_block();
  const int row0 = lb * BS;
  const int t = threadIdx.x;
  const bool mine = row0 + t < a.n;
  const int row = mine ? row0 + t : 0;
  const double pv = a.p[q][row], vv = a.v[q][row], xv = a.x[row], rv = a.r[row];
  const double tv = a.t[row], rhv = a.rh[row], wv = a.W ? a.W[row] : 0.0;
  asm volatile("" ::: "memory");
  if (st != ST_RUNNING && st != ST_HALF) return;
  mark_work(c, a.pslot, 8.0 * a.n * (st == ST_HALF ? 3 : (a.W ? 9 : 8)));
  if (st == ST_HALF) {
    if (mine) a.x[row] = fma(alpha, pv, xv);
    return;
  }
  double acc[3] = {0.0, 0.0, 0.0};
  if (mine) {
    const double s = fma(-alpha, vv, rv);
    a.x[row] = fma(omega, s, fma(alpha, pv, xv));
    const double r = fma(-omega, tv, s);
    a.r[row] = r;
    acc[0] = rhv * r;
    acc[1] = r * r;
    if (a.W) {
      const double wr = wv * r;
      acc[2] = wr * wr;
    }
  }
  block_partials<3>(acc, 3, a.partials, nb, lb, red);
}

// FU: stop test on ||W r|| (or the iteration cap), then rho, beta, or breakdown.
template <bool BIG>
__global__ __launch_bounds__(BS) void k_bicg_fin_u(Ctl* c, const double* partials, int nb,
                                                   int has_w) {
  const int st = c->sum.state, iters = c->sum.iters, maxit = c->maxit;
  const double ref = c->ref, tol = c->tol, eps_b = c->eps_b, rh_norm = c->rh_norm;
  const double rho = c->rho, alpha = c->alpha, omega = c->omega;
  __shared__ double out[8];
  if constexpr (BIG) {
    if (!split_sums<3, sum_batch<3>()>(c, partials, nb, out)) return;
  } else {
    small_sums<3, SUM_BATCH>(partials, nb, out);
  }
  if (threadIdx.x != 0) return;
  if (st == ST_HALF) {
    c->sum.state = ST_VERIFY;
    return;
  }
  if (st != ST_RUNNING) return;
  const double rn = sqrt(out[1]);
  const double est = (has_w ? sqrt(out[2]) : rn) / ref;
  c->sum.relres_rec = est;
  if (est < tol || iters >= maxit) {
    c->sum.state = ST_VERIFY;
    return;
  }
  const double rho_new = out[0];
  if (fabs(rho_new) <= eps_b * rh_norm * rn) {
    c->sum.status = S_BREAKDOWN;
    c->sum.brk = BRK_RHO;
    c->sum.state = ST_FINAL;
    return;
  }
  c->beta = (rho_new / rho) * (alpha / omega);
  c->rho_old = rho;
  c->rho = rho_new;
  c->first = 0;
}

template <class Op>
static void launch_residual(const BArgs& a, const Op& op, int nb, const int* flags,
                            hipStream_t s, bool probe = true) {
  BArgs ax = a;
  ax.pslot = probe ? probe_slot(KC_RESIDUAL) : -1;
  launch_probed(k_bicg_residual<Op>, dim3(nb), s, ax.pslot, ax, op, flags);
  hipLaunchKernelGGL(k_bicg_fin_residual, dim3(1), dim3(BS), 0, s, a.ctl,
                     (const double*)a.partials, nb, a.W ? 1 : 0, flags);
}

template <class Op>
static void launch_iteration(const BArgs& a, const Op& op, int nb, int par, hipStream_t s,
                             bool probe = true) {
  const int hw = a.W ? 1 : 0;
  const double* pt = a.partials;
  BArgs ax = a;
  ax.par = par;
  // the window kernels for large systems; small ones are bound by launch latency, where the
  // one-tile kernels' speculative loads are faster (the bits are the same either way)
  bool window = false;
  if constexpr (std::is_same_v<Op, StencilOp>)
    window = op.ldp == (size_t)op.n && op.nx <= WIN_NX && op.n >= kWindowRows;
  const dim3 gw(grid_for(a.n, 2));
  ax.pslot = probe ? probe_slot(KC_BICG_P) : -1;
  if constexpr (std::is_same_v<Op, StencilOp>) {
    if (window) launch_probed(k_bicg_p_win, gw, s, ax.pslot, ax, op, nb);
    else launch_probed(k_bicg_p<Op>, dim3(nb), s, ax.pslot, ax, op);
  } else {
    launch_probed(k_bicg_p<Op>, dim3(nb), s, ax.pslot, ax, op);
  }
  // systems of many tiles: finalize launches split over WAVES workgroups, with larger
  // batches of partials (the same sums)
  const bool big = nb > SUM_BATCH * BS;
  const dim3 fg(big ? WAVES : 1), fb(big ? 64 : BS);
  hipLaunchKernelGGL(big ? k_bicg_fin_p<true> : k_bicg_fin_p<false>, fg, fb, 0, s, a.ctl, pt,
                     nb);
  ax.pslot = probe ? probe_slot(KC_BICG_S) : -1;
  if constexpr (std::is_same_v<Op, StencilOp>) {
    if (window) launch_probed(k_bicg_s_win, gw, s, ax.pslot, ax, op, nb);
    else launch_probed(k_bicg_s<Op>, dim3(nb), s, ax.pslot, ax, op);
  } else {
    launch_probed(k_bicg_s<Op>, dim3(nb), s, ax.pslot, ax, op);
  }
  hipLaunchKernelGGL(big ? k_bicg_fin_s<true> : k_bicg_fin_s<false>, fg, fb, 0, s, a.ctl, pt,
                     nb, hw);
  ax.pslot = probe ? probe_slot(KC_BICG_U) : -1;
  launch_probed(k_bicg_u, dim3(nb), s, ax.pslot, ax);
  hipLaunchKernelGGL(big ? k_bicg_fin_u<true> : k_bicg_fin_u<false>, fg, fb, 0, s, a.ctl, pt,
                     nb, hw);
}

static SolveResult bfail(int code) {
  SolveResult r;
  r.code = code;
  r.sum = Summary{};
  return r;
}

// Without allocation (noalloc): the workspace is the caller's (here the file-scope scratch
// array), status is read with a copy into host stack memory and a stream synchronisation per
// chunk (no pinned memory, no events), and no launch is timed by the measurement hook. The
// launches, and so the results, are those of the ordinary path.
template <class Op>
static SolveResult bicgstab_run_noalloc(const Mat& A, const Op& op, const BArgs& a,
                                        const Workspace& Wk, const Geom& g,
                                        const SolveParams& prm, hipStream_t s) {
  SolveResult res;
  res.code = 0;
  res.sum = Summary{};
  const int k = prm.check_every;
  Pacer pace{prm.tol, prm.maxit, k};
  if ((long)2 * k >= prm.maxit) pace.cautious = true;
  long launched = 0;
  Summary sum{};
  const long max_chunks = (long)prm.maxit * 4 + 16;
  bool done = false;
  for (long ch = 0; ch <= max_chunks && !done; ++ch) {
    const int count = pace.cautious && k > 1 ? k / 2 : k;
    for (int it = 0; it < count; ++it, ++launched)
      launch_iteration(a, op, g.nb, (int)(launched & 1), s, false);
    launch_residual(a, op, g.nb, Wk.flags, s, false);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&sum, &Wk.ctl->sum, sizeof(Summary), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      res.code = -5;
      return res;
    }
    if (sum.state == ST_DONE) done = true;
    else pace.update(sum.iters, sum.relres_rec);
  }
  res.sum = sum;
  if (!done) res.code = -5;
  else if (sum.status < 0) res.code = -1;
  return res;
}

template <class Op>
static SolveResult bicgstab_run(const Mat& A, const Op& op, const double* b, double* x,
                                const SolveParams& prm, void* ws, hipStream_t s,
                                bool noalloc = false) {
  Workspace Wk = carve(ws, A.n);
  const Geom g = make_geom(A.n);
  const size_t ld = vec_ld(A.n);
  double* base = Wk.vecs;
  BArgs a;
  a.n = A.n;
  a.rpb = g.rpb;
  a.ctl = Wk.ctl;
  a.partials = Wk.partials;
  a.r = base;
  a.rh = base + ld;
  a.p[0] = base + 2 * ld;
  a.p[1] = base + 3 * ld;
  a.v[0] = base + 4 * ld;
  a.v[1] = base + 5 * ld;
  a.t = base + 6 * ld;
  a.x = x;
  a.b = b;
  a.W = prm.weights;
  a.mat_bytes = A.bytes();
  a.pslot = -1;
  a.par = 0;
  if (launch_clear_flags(Wk.flags, s) != hipSuccess) return bfail(-5);
  if (A.kind == MAT_CSR && launch_validate(A.csr, Wk.flags, s) != hipSuccess) return bfail(-5);
  hipLaunchKernelGGL(k_bicg_init_ctl, dim3(1), dim3(64), 0, s, Wk.ctl, prm.maxit, prm.tol,
                     prm.eps_b, prm.weights ? 1 : 0);
  if (noalloc) {
    launch_residual(a, op, g.nb, Wk.flags, s, false);
    if (hipGetLastError() != hipSuccess) return bfail(-5);
    return bicgstab_run_noalloc(A, op, a, Wk, g, prm, s);
  }
  probe_solve_begin();
  launch_residual(a, op, g.nb, Wk.flags, s);
  if (hipGetLastError() != hipSuccess) return bfail(-5);

  Summary* hs = pinned_summaries();
  if (!hs) return bfail(-5);
  hipEvent_t ev[2];
  if (hipEventCreateWithFlags(&ev[0], hipEventDisableTiming) != hipSuccess) return bfail(-5);
  if (hipEventCreateWithFlags(&ev[1], hipEventDisableTiming) != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return bfail(-5);
  }
  SolveResult res;
  res.code = 0;
  int slot = 0;
  bool pending = false, done = false;
  const int k = prm.check_every;
  Pacer pace{prm.tol, prm.maxit, k};
  if ((long)2 * k >= prm.maxit) pace.cautious = true;
  long launched = 0;   // iterations enqueued so far: gives each its buffer parity
  auto chunk = [&](int count) {
    for (int it = 0; it < count; ++it, ++launched)
      launch_iteration(a, op, g.nb, (int)(launched & 1), s);
    launch_residual(a, op, g.nb, Wk.flags, s);
    return hipGetLastError() == hipSuccess;
  };
  auto record = [&](int sl) {
    return hipMemcpyAsync(&hs[sl], &Wk.ctl->sum, sizeof(Summary), hipMemcpyDeviceToHost, s) ==
               hipSuccess &&
           hipEventRecord(ev[sl], s) == hipSuccess;
  };
  auto check = [&](int sl) {
    if (hipEventSynchronize(ev[sl]) != hipSuccess) return false;
    if (hs[sl].state == ST_DONE) done = true;
    else pace.update(hs[sl].iters, hs[sl].relres_rec);
    return true;
  };
  // Every chunk either advances the iteration count or finishes; bound the loop generously.
  const long max_chunks = (long)prm.maxit * 4 + 16;
  for (long ch = 0; ch <= max_chunks && !done; ++ch) {
    if (!pace.cautious) {
      // Enqueue a chunk, then read the previous chunk's status while it runs.
      if (!chunk(k) || !record(slot)) { res.code = -5; break; }
      if (pending && !check(slot ^ 1)) { res.code = -5; break; }
      pending = true;
      slot ^= 1;
      continue;
    }
    if (pending) {   // first wait for the chunk still in flight
      if (!check(slot ^ 1)) { res.code = -5; break; }
      pending = false;
      if (done) break;
    }
    // Near the end: half chunks, each waited for before the next is enqueued.
    if (!chunk(k > 1 ? k / 2 : 1) || !record(slot) || !check(slot)) { res.code = -5; break; }
    slot ^= 1;
  }
  if (hipStreamSynchronize(s) != hipSuccess && res.code == 0) res.code = -5;
  if (res.code == 0) probe_collect(&Wk.ctl->probe, s);
  if (res.code == 0) {
    res.sum = hs[slot ^ 1];
    if (res.sum.state != ST_DONE) res.code = -5;
    else if (res.sum.status < 0) res.code = -1;
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  return res;
}

SolveResult bicgstab_solve(const Mat& A, const double* b, double* x, const SolveParams& prm,
                           void* ws, hipStream_t s) {
  if (A.kind == MAT_STENCIL) return bicgstab_run(A, A.stencil_op(), b, x, prm, ws, s);
  return bicgstab_run(A, A.csr_op(), b, x, prm, ws, s);
}

// ---------------------------------------------------------------------------------------
// Bi-CGSTAB without allocation (gsk_bicgstab_noalloc): the workspace is a file-scope device
// array of kNoAllocBytes, one per GPU the library runs on, held until the process ends. Its
// name is a host-side stand-in in host code; the device address of each GPU's copy is looked
// up once per device (hipGetSymbolAddress, with that device current) and only that address
// is handed to the kernels. Every call on a GPU shares that GPU's array and leaves its
// contents behind; the solver initialises everything it reads (control block by its init
// kernel, flags by a clear kernel, partials and vectors by the launches that produce them),
// so nothing has to start at zero. Calls that overlap on one GPU race on the array.
// ---------------------------------------------------------------------------------------
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// The current device's copy of scratch (looked up on the first call on that device), or
// nullptr with *err set.
void* noalloc_scratch(hipError_t* err) {
  int dev = 0;
  *err = hipGetDevice(&dev);
  if (*err != hipSuccess) return nullptr;
  if (dev < 0 || dev >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (*err != hipSuccess || !ptr) {
      if (*err == hipSuccess) *err = hipErrorInvalidSymbol;
      return nullptr;
    }
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

SolveResult bicgstab_solve_noalloc(const Mat& A, const double* b, double* x,
                                   const SolveParams& prm, void* scratch_ptr, hipStream_t s) {
  if (A.kind == MAT_STENCIL)
    return bicgstab_run(A, A.stencil_op(), b, x, prm, scratch_ptr, s, true);
  return bicgstab_run(A, A.csr_op(), b, x, prm, scratch_ptr, s, true);
}

}  // namespace gsk
