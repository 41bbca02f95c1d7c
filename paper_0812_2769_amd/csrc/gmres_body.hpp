// Workgroup bodies of the GMRES(m) kernels, shared by the single solver (gmres.hip, one system
// over the whole grid) and the batch engine (batch_gmres.hip, many systems, each workgroup on
// one system's rows). Each body works on the rows of one workgroup index lb of one system and
// writes its partial sums to partials[col * pstride + lb]; the finalize bodies reduce `count`
// such partials of one system. Whoever calls them, the arithmetic and its order are the same,
// so a system gives the same bits in the batch as alone. The algorithm is described in
// gmres.hip.
#pragma once

#include "gsk_dev.hpp"

namespace gsk {

__device__ inline int tile_rows(int n, int row0) { return max(0, min(BS, n - row0)); }

// Workgroup total of one per-thread value into partials[col * pstride + lb].
__device__ inline void block_single_partial(double v, double* __restrict__ partials, int col,
                                            int pstride, int lb, double* lds) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < WAVES; ++q) s += lds[q];
    partials[(size_t)col * pstride + lb] = s;
  }
}

// Rows per thread. A workgroup owns RPT consecutive tiles of BS rows and thread t the rows
// row0 + q BS + t, q < RPT. FP32 data use RPT = 2, so that a thread keeps as many bytes of
// loads in flight as an FP64 thread; a CSR product stages one tile at a time through LDS and
// keeps RPT = 1.
template <class T>
constexpr int rpt_of() { return 8 / (int)sizeof(T); }

// (double)x for a value the kernel has already widened once. The empty asm makes the two
// conversions distinct to the compiler, so it keeps the narrow value (one register for a
// float) alive instead of the widened one (two registers), which would halve occupancy.
template <class T>
__device__ inline double widen_again(T x) {
  if constexpr (sizeof(T) == 4) asm("" : "+v"(x));
  return (double)x;
}

// R (tile lb): r = b - A x (FP64) into u_0 stored as T; partials ||r||^2 (column 0),
// ||W r||^2 (column 1) and ||u_0||^2 of the stored values (column 2). bad != 0: the system's
// data were rejected and nothing is computed.
template <class Op, class T>
__device__ inline void gmres_residual_tile(Ctl* c, const Op& op, int n,
                                           const double* __restrict__ b,
                                           const double* __restrict__ x,
                                           const double* __restrict__ W, T* __restrict__ u0,
                                           int bad, int lb, double* __restrict__ partials,
                                           int pstride, int pslot, double mat_bytes,
                                           typename Op::Lds& L, double* red) {
  const int st = c->sum.state;
  if (st != ST_INIT && st != ST_CYCLE_END) return;
  if (bad) return;
  mark_work(c, pslot, mat_bytes + n * (16.0 + sizeof(T) + (W ? 8.0 : 0.0)));
  const int row0 = lb * BS;
  const int nrows = tile_rows(n, row0);
  double acc[3] = {0.0, 0.0, 0.0};
  if (nrows > 0) {
    const double y = op.tile(row0, nrows, GatherX{x}, L);
    if ((int)threadIdx.x < nrows) {
      const int row = row0 + threadIdx.x;
      const double r = b[row] - y;
      const T rs = (T)r;
      u0[row] = rs;
      acc[0] = r * r;
      if (W) {
        const double wr = W[row] * r;
        acc[1] = wr * wr;
      }
      acc[2] = (double)rs * (double)rs;
    }
  }
  block_partials<3>(acc, 3, partials, pstride, lb, red);
}

// FR: convergence / restart decision after the true residual (see gmres.hip). The partials
// of the residual body are at partials[col * pstride + l], l < count. bad < 0 ends the solve
// with that status.
__device__ inline void gmres_fin_residual_body(Ctl* c, const double* partials, int count,
                                               int pstride, int has_w, int mixed, int bad) {
  const int st = c->sum.state;
  if (st != ST_INIT && st != ST_CYCLE_END) return;
  if (bad) {
    if (threadIdx.x == 0) {
      c->sum.state = ST_DONE;
      c->sum.status = bad;
    }
    return;
  }
  __shared__ double out[8];
  small_sums_strided<3>(partials, count, pstride, out);
  if (threadIdx.x != 0) return;
  const double nr = sqrt(out[0]);
  const double nwr = has_w ? sqrt(out[1]) : nr;
  const double ns = sqrt(out[2]);   // norm of the stored u_0 (equals nr in FP64)
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
    if (c->broke) {
      c->sum.status = S_BREAKDOWN;
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
    const int progress = mixed && rt < 0.5 * c->last_rt;
    if (c->claimed && !progress) {
      c->sum.fails += 1;
      if (c->sum.fails >= 3) {
        c->sum.status = S_STAGNATED;
        c->sum.state = ST_DONE;
        return;
      }
    } else {
      c->sum.fails = 0;
    }
    c->sum.restarts += 1;
  }
  // start a cycle: v_0 = u_0 / ||u_0||, g = ||u_0|| e_1; the cycle's estimates are in the
  // norm of the stored u_0 and are converted to the stop-test metric by nwr / ns
  c->last_rt = nwr / c->ref;
  c->sigma[0] = 1.0 / ns;
  c->g[0] = ns;
  for (int i = 1; i <= c->m; ++i) c->g[i] = 0.0;
  c->ratio = nwr / ns;
  c->j = 0;
  c->k = 0;
  c->claimed = 0;
  c->happy = 0;
  c->sum.state = ST_RUNNING;
}

// A (workgroup lb, RPT tiles): w = A u_j of the stored (unnormalised) column, so that A
// needs no scalar of step j-1 (sigma_j enters the finalize launches and C instead); partials
// of u_i . w (columns 0..j) and ||w||^2 (column j+1). Loads are issued in the order they are
// needed (stencil operands, then the basis values of the thread's rows) before the body tests
// whether it has work: the control block is read alongside, so the test costs no round trip
// of its own. The step runs while the solve runs and its step counter reads jexp: j when the
// finalize of step j-1 has run, j-1 when it runs later (the single solver's merged launch,
// which discards this step's sums if step j-1 ends the cycle). A body without work stores
// nothing.
template <int JM, int RPT, class R, class Op, class T>
__device__ inline void gmres_a_tile(Ctl* c, const Op& op, int n, const T* __restrict__ V,
                                    size_t ldv, T* __restrict__ w, int j, int jexp, int lb,
                                    double* __restrict__ partials, int pstride, T zero,
                                    int pslot, double inner_bytes, typename Op::Lds& L,
                                    double* red, double* red1) {
  const int state = c->sum.state, cj = c->j;
  const int t = threadIdx.x;
  const GatherXT<T> gx{V + (size_t)j * ldv};
  const R rd(V, ldv, j + 1);
  int rq[RPT], nq[RPT];
  typename Op::template Pre<GatherXT<T>> pre[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    rq[q] = (lb * RPT + q) * BS;
    nq[q] = tile_rows(n, rq[q]);
    pre[q] = op.load(rq[q], nq[q], gx);   // unconditional: valid rows for any tile
  }
  T u[JM][RPT];
#pragma unroll
  for (int i = 0; i < JM; ++i)
#pragma unroll
    for (int q = 0; q < RPT; ++q)
      u[i][q] = (i <= j && t < nq[q]) ? rd.raw(i, rq[q] + t) : zero;
  // A CSR product follows the row pointers and column indices, which are trusted only while
  // the solve runs (structure rejected by validation ends it): test first. A stencil product
  // reads clamped addresses only and goes ahead of the test.
  if constexpr (!Op::kRowwise) {
    if (state != ST_RUNNING || cj != jexp) return;
  }
  double y[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) y[q] = nq[q] > 0 ? op.finish(pre[q], rq[q], nq[q], gx, L) : 0.0;
  asm volatile("" ::: "memory");   // keeps the loads above ahead of the test below
  if (state != ST_RUNNING || cj != jexp) return;
  mark_work(c, pslot, inner_bytes + (double)sizeof(T) * n * (j + 2));
  double wr[RPT], nrm = 0.0;
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const T ws = (T)y[q];
    const bool mine = t < nq[q];
    wr[q] = mine ? (double)ws : 0.0;
    if (mine) w[rq[q] + t] = ws;
    nrm += wr[q] * wr[q];
  }
  double v[JM];
#pragma unroll
  for (int i = 0; i < JM; ++i) {
    v[i] = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) v[i] += widen_again(u[i][q]) * wr[q];
  }
  block_halving_partials<JM>(v, j + 1, partials, pstride, lb, red);
  block_single_partial(nrm, partials, j + 1, pstride, lb, red1);
}

// FA (one workgroup per column col): col <= j -> c1_col = sigma_col (u_col . w), the pass-1
// coefficient in the scale of w = A u_j (the Hessenberg entry is sigma_j c1_col), and its
// update weight d1_col = c1_col sigma_col; col = j+1 -> ||w||. `col_partials` is that column's
// `count` partials. The control words are read together with the partials (one memory round
// trip) and only the store depends on them.
// kMerged: the single solver's launch that also runs FC of step j-1 (in another workgroup),
// which writes sigma_j, the step counter and the state while this body runs. The body then
// reads none of them: column j computes sigma_j itself from C's `ccount` partials `cpart`,
// with FC's arithmetic, and the stores are unconditional (if step j-1 ends the cycle, nothing
// reads them before the next cycle rewrites them).
template <bool kMerged = false, int SB = SUM_BATCH>
__device__ inline void gmres_fin_a_body(Ctl* c, const double* col_partials, int count, int j,
                                        int col, double* lds, const double* cpart = nullptr,
                                        int ccount = 0) {
  int state = ST_RUNNING, cj = j;
  if constexpr (!kMerged) {
    state = c->sum.state;
    cj = c->j;
  }
  const bool own = kMerged && col == j;
  const double sg0 = (col <= j && !own) ? c->sigma[col] : 0.0;
  const double s = column_sum<SB>(col_partials, count, lds);
  const double sg = own ? 1.0 / sqrt(column_sum<SB>(cpart, ccount, lds)) : sg0;
  if (state != ST_RUNNING || cj != j || threadIdx.x != 0) return;
  const int par = j & 1;
  if (col == j + 1) {
    c->wnorm_pre[par] = sqrt(s);
  } else {
    const double c1 = sg * s;
    c->c1[par][col] = c1;
    c->d1[col] = c1 * sg;
  }
}

// B: w -= sum_i c1_i v_i (weights d1_i = c1_i sigma_i on the stored columns), then partials of
// u_i . w, sharing one read of the basis. Operands are requested before the work test, as in A.
template <int JM, int RPT, class R, class T>
__device__ inline void gmres_b_tile(Ctl* c, int n, const T* __restrict__ V, size_t ldv,
                                    T* __restrict__ w, int j, int lb,
                                    double* __restrict__ partials, int pstride, T zero,
                                    int pslot, double* red) {
  const int state = c->sum.state, cj = c->j;
  const int t = threadIdx.x;
  double d[JM];   // uniform across the launch: scalar loads
#pragma unroll
  for (int i = 0; i < JM; ++i) d[i] = c->d1[i];
  const R rd(V, ldv, j + 1);
  int row[RPT];
  bool mine[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    row[q] = (lb * RPT + q) * BS + t;
    mine[q] = row[q] < n;
  }
  T u[JM][RPT];
#pragma unroll
  for (int i = 0; i < JM; ++i)
#pragma unroll
    for (int q = 0; q < RPT; ++q) u[i][q] = (i <= j && mine[q]) ? rd.raw(i, row[q]) : zero;
  T wv[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) wv[q] = mine[q] ? w[row[q]] : zero;
  asm volatile("" ::: "memory");
  if (state != ST_RUNNING || cj != j) return;
  mark_work(c, pslot, (double)sizeof(T) * n * (j + 3));
  double wr[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    double x = (double)wv[q];
#pragma unroll
    for (int i = 0; i < JM; ++i)
      if (i <= j) x = fma(-d[i], (double)u[i][q], x);
    const T ws = (T)x;
    wr[q] = mine[q] ? (double)ws : 0.0;
    if (mine[q]) w[row[q]] = ws;
  }
  double v[JM];
#pragma unroll
  for (int i = 0; i < JM; ++i) {
    v[i] = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) v[i] += widen_again(u[i][q]) * wr[q];
  }
  block_halving_partials<JM>(v, j + 1, partials, pstride, lb, red);
}

// FB (one workgroup per column col <= j): c2_col = sigma_col (u_col . w).
template <int SB = SUM_BATCH>
__device__ inline void gmres_fin_b_body(Ctl* c, const double* col_partials, int count, int j,
                                        int col, double* lds) {
  const int state = c->sum.state, cj = c->j;
  const double sg = c->sigma[col];
  const double s = column_sum<SB>(col_partials, count, lds);
  if (state != ST_RUNNING || cj != j || threadIdx.x != 0) return;
  const double c2 = sg * s;
  c->c2[col] = c2;
  c->d2[col] = c2 * sg;
}

// C: w -= sum_i c2_i v_i (weights d2_i = c2_i sigma_i), u_{j+1} = sigma_j w (back in the
// scale of v_j, so that the stored columns keep norms of the order of the Hessenberg entries),
// partial ||u_{j+1}||^2. Operands are requested before the work test, as in A.
template <int JM, int RPT, class R, class T>
__device__ inline void gmres_c_tile(Ctl* c, int n, T* __restrict__ V, size_t ldv,
                                    const T* __restrict__ w, int j, int lb,
                                    double* __restrict__ partials, int pstride, T zero,
                                    int pslot, double* red) {
  const int state = c->sum.state, cj = c->j;
  const double sg = c->sigma[j];
  const int t = threadIdx.x;
  double d[JM];   // uniform across the launch: scalar loads
#pragma unroll
  for (int i = 0; i < JM; ++i) d[i] = c->d2[i];
  const R rd(V, ldv, j + 1);
  int row[RPT];
  bool mine[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    row[q] = (lb * RPT + q) * BS + t;
    mine[q] = row[q] < n;
  }
  T u[JM][RPT];
#pragma unroll
  for (int i = 0; i < JM; ++i)
#pragma unroll
    for (int q = 0; q < RPT; ++q) u[i][q] = (i <= j && mine[q]) ? rd.raw(i, row[q]) : zero;
  T wv[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) wv[q] = mine[q] ? w[row[q]] : zero;
  asm volatile("" ::: "memory");
  if (state != ST_RUNNING || cj != j) return;
  mark_work(c, pslot, (double)sizeof(T) * n * (j + 3));
  double nrm = 0.0;
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    double x = (double)wv[q];
#pragma unroll
    for (int i = 0; i < JM; ++i)
      if (i <= j) x = fma(-d[i], (double)u[i][q], x);
    const T ws = (T)(sg * x);
    const double wr = mine[q] ? (double)ws : 0.0;
    if (mine[q]) V[(size_t)(j + 1) * ldv + row[q]] = ws;
    nrm += wr * wr;
  }
  block_single_partial(nrm, partials, 0, pstride, lb, red);
}

// FC (one workgroup): Hessenberg column (h_ij = sigma_j (c1_i + c2_i), h_{j+1,j} = ||u_{j+1}||),
// Givens rotations, residual estimate; at the end of a cycle the k x k triangular solve
// H y = g (y stored pre-multiplied by sigma). `partials` are the `count` partials of C. Every control word the body needs is requested before the first
// wait; the old rotations are applied in registers by one thread.
template <int SB = SUM_BATCH>
__device__ inline void gmres_fin_c_body(Ctl* c, const double* partials, int count, int j) {
  __shared__ double lds[WAVES];
  __shared__ double s_h[MMAX + 2];
  __shared__ double s_cs[MMAX], s_sn[MMAX];
  __shared__ int s_end, s_k;
  constexpr int LDH = MMAX + 1;
  const int t = threadIdx.x;
  const int state = c->sum.state, cj = c->j;
  const int iters = c->sum.iters, maxit = c->maxit, m = c->m;
  const int par = j & 1;
  const double sgj = c->sigma[j];
  const double eps_b = c->eps_b, wpre = sgj * c->wnorm_pre[par], gj = c->g[j];
  const double ratio = c->ratio, ref = c->ref, tol = c->tol;
  if (t <= j) {
    s_h[t] = (c->c1[par][t] + c->c2[t]) * sgj;
    s_cs[t] = c->cs[t];
    s_sn[t] = c->sn[t];
  }
  const double nrm2 = column_sum<SB>(partials, count, lds);   // also orders the LDS writes above
  if (state != ST_RUNNING || cj != j) return;
  const double hn = sqrt(nrm2);
  if (t <= j) c->Hraw[(size_t)j * LDH + t] = s_h[t];
  if (t == j + 1) c->Hraw[(size_t)j * LDH + t] = hn;
  if (t == 0) {
    const int happy = hn <= eps_b * wpre;
    c->happy = happy;
    if (!happy) c->sigma[j + 1] = 1.0 / hn;
    double hi = s_h[0];
    for (int i = 0; i < j; ++i) {
      const double hnext = s_h[i + 1];
      s_h[i] = s_cs[i] * hi + s_sn[i] * hnext;
      hi = -s_sn[i] * hi + s_cs[i] * hnext;
    }
    const double dd = hypot(hi, hn);
    c->sum.iters = iters + 1;
    int end = 0, k = j + 1;
    if (dd == 0.0) {
      c->broke = 1;
      c->sum.brk = BRK_GIVENS;
      k = j;
      end = 1;
      s_h[j] = hi;
      s_h[j + 1] = hn;
    } else {
      const double cjr = hi / dd;
      const double sjr = hn / dd;
      s_h[j] = dd;
      s_h[j + 1] = 0.0;
      const double g1 = -sjr * gj;
      c->g[j + 1] = g1;
      c->g[j] = cjr * gj;
      c->cs[j] = cjr;
      c->sn[j] = sjr;
      const double est = fabs(g1) * ratio / ref;
      c->sum.relres_rec = est;
      const int claimed = (est < tol) || happy;
      c->claimed = claimed;
      end = claimed || (iters + 1 >= maxit) || (j + 1 == m);
    }
    c->j = j + 1;
    c->k = k;
    s_end = end;
    s_k = k;
  }
  __syncthreads();
  if (t <= j + 1) c->H[(size_t)j * LDH + t] = s_h[t];
  if (!s_end) return;

  __shared__ double s_H[MMAX][MMAX + 1];   // s_H[col][row]
  __shared__ double s_g[MMAX + 1], s_y[MMAX];
  const int k = s_k;
  for (int idx = t; idx < k * k; idx += BS) {
    const int col = idx / k, row = idx % k;
    s_H[col][row] = (col == j) ? s_h[row] : c->H[(size_t)col * LDH + row];
  }
  if (t < k) s_g[t] = c->g[t];
  __syncthreads();
  for (int i = k - 1; i >= 0; --i) {
    if (t == 0) s_y[i] = s_g[i] / s_H[i][i];
    __syncthreads();
    if (t < i) s_g[t] -= s_H[i][t] * s_y[i];
    __syncthreads();
  }
  if (t < k) c->y[t] = s_y[t] * c->sigma[t];
  __syncthreads();
  if (t == 0) c->sum.state = ST_CYCLE_END;
}

// X (workgroup lb, RPT tiles): x += sum_{l<k} y_l v_l (y already carries sigma).
template <int RPT, class R, class T>
__device__ inline void gmres_x_tile(Ctl* c, int n, const T* __restrict__ V, size_t ldv,
                                    double* __restrict__ x, int lb, int pslot, double* s_y) {
  if (c->sum.state != ST_CYCLE_END) return;
  const int k = c->k;
  mark_work(c, pslot, n * ((double)sizeof(T) * k + 16.0));
  const int t = threadIdx.x;
  if (t < k) s_y[t] = c->y[t];
  __syncthreads();
  const R rd(V, ldv, k > 0 ? k : 1);
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int row = (lb * RPT + q) * BS + t;
    if (row >= n) continue;
    double acc = 0.0;
    for (int l = 0; l < k; ++l) acc = fma(s_y[l], rd.load(l, row), acc);
    x[row] = x[row] + acc;
  }
}

}  // namespace gsk
