// Restarted GMRES(m) with double classical Gram-Schmidt (CGS2) Arnoldi, and the bare
// Arnoldi process, on the device.
//
// Section 2 of the paper: restarted GMRES whose Arnoldi step orthogonalises with a double
// classical Gram-Schmidt pass. One Arnoldi step j (basis columns u_0..u_j stored unnormalised
// with scale factors sigma_i, so v_i = sigma_i u_i) is three streaming launches, each
// followed by a small finalize launch that reduces the per-workgroup partials:
//
//   A  w = A v_j (CSR tile product), partial c1 = V_j^T w, ||w||^2   reads A, V_j; writes w
//      FA: c1_i, ||A v_j||                                          (j+2 workgroups)
//   B  w -= V_j c1, partial c2 = V_j^T w                             reads V_j, w; writes w
//      FB: c2_i                                                     (j+1 workgroups)
//   C  w -= V_j c2, u_{j+1} = w, partial ||w||^2                     reads V_j, w; writes u
//      FC: h_{j+1,j}, Givens rotations, residual estimate, and at the end of a cycle the
//          triangular solve for y                                   (1 workgroup)
//
// The basis is read three times per step instead of four: the update of pass 1 and the dot
// products of pass 2 share one read, with the basis values held in registers. The division
// v_{j+1} = w / h_{j+1,j} is never materialised: sigma_{j+1} = 1/h_{j+1,j} is folded into the
// coefficients of later passes. At the end of a cycle X adds V_k y to x and R (+ FR)
// recomputes the true residual r = b - A x, which either ends the solve or starts the next
// cycle with u_0 = r.
//
// Every launch first checks the device-resident state and returns at once if the solve has
// moved on, so a whole cycle can be enqueued (or replayed from a graph) blindly; the host
// reads a small summary once per cycle.
#include "gsk_host.hpp"

namespace gsk {

struct KArgs {
  int n;
  int rpb;
  Ctl* ctl;
  double* partials;
  double mat_bytes;   // algorithmic bytes of one read of A (CSR: 12 nnz + 4 (n+1))
  int pslot;          // measurement slot of this launch, or -1
};

__global__ __launch_bounds__(64) void k_init_ctl(Ctl* c, int maxit, int m, double tol,
                                                 double eps_b, int has_w) {
  for (int i = threadIdx.x; i < PROBE_SLOTS; i += 64) c->probe.bytes[i] = 0.0;
  if (threadIdx.x != 0) return;
  c->sum.state = ST_INIT;
  c->sum.status = S_MAXIT;
  c->sum.iters = 0;
  c->sum.restarts = 0;
  c->sum.half = 0;
  c->sum.fails = 0;
  c->sum.steps = 0;
  c->sum.brk = BRK_NONE;
  c->sum.relres_rec = 1.0;
  c->sum.relres_true = 1.0;
  c->maxit = maxit;
  c->m = m;
  c->j = 0;
  c->k = 0;
  c->claimed = 0;
  c->first = 1;
  c->has_w = has_w;
  c->broke = 0;
  c->happy = 0;
  c->tol = tol;
  c->eps_b = eps_b;
  c->ref = 0.0;
  c->ratio = 1.0;
  c->rho = c->rho_old = c->alpha = c->omega = c->beta = c->rh_norm = 0.0;
  c->wnorm_pre = 0.0;
}

// Every streaming kernel below works on one tile of BS rows per workgroup, one row per
// thread (workgroup lb of the XCD-aware numbering owns rows [lb*BS, lb*BS + BS)).
__device__ inline int tile_rows(int n, int row0) { return max(0, min(BS, n - row0)); }

// Workgroup total of one per-thread value into partials[col * nb + lb].
__device__ inline void block_single_partial(double v, double* __restrict__ partials, int col,
                                            int nb, int lb, double* lds) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < WAVES; ++q) s += lds[q];
    partials[(size_t)col * nb + lb] = s;
  }
}

// R: r = b - A x into u_0; partials ||r||^2 (column 0), ||W r||^2 (column 1).
template <class Op>
__global__ __launch_bounds__(BS) void k_gmres_residual(KArgs a, Op op, const double* __restrict__ b,
                                                       const double* __restrict__ x,
                                                       const double* __restrict__ W,
                                                       double* __restrict__ u0,
                                                       const int* flags) {
  Ctl* c = a.ctl;
  const int st = c->sum.state;
  if (st != ST_INIT && st != ST_CYCLE_END) return;
  if (flags[0]) return;
  mark_work(c, a.pslot, a.mat_bytes + 8.0 * a.n * (W ? 4 : 3));
  __shared__ typename Op::Lds L;
  __shared__ double red[NC_MAX * WAVES];
  const int nb = gridDim.x;
  const int lb = logical_block();
  const int row0 = lb * BS;
  const int nrows = tile_rows(a.n, row0);
  double acc[2] = {0.0, 0.0};
  if (nrows > 0) {
    const double y = op.tile(row0, nrows, GatherX{x}, L);
    if ((int)threadIdx.x < nrows) {
      const int row = row0 + threadIdx.x;
      const double r = b[row] - y;
      u0[row] = r;
      acc[0] = r * r;
      if (W) {
        const double wr = W[row] * r;
        acc[1] = wr * wr;
      }
    }
  }
  block_partials<2>(acc, 2, a.partials, nb, lb, red);
}

// FR: convergence / restart decision after the true residual (see file comment).
__global__ __launch_bounds__(BS) void k_gmres_fin_residual(Ctl* c, const double* partials,
                                                           int nb, int has_w,
                                                           const int* flags) {
  const int st = c->sum.state;
  if (st != ST_INIT && st != ST_CYCLE_END) return;
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
    if (c->claimed) {
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
  // start a cycle: v_0 = r / ||r||, g = ||r|| e_1
  c->sigma[0] = 1.0 / nr;
  c->g[0] = nr;
  for (int i = 1; i <= c->m; ++i) c->g[i] = 0.0;
  c->ratio = has_w ? nwr / nr : 1.0;
  c->j = 0;
  c->k = 0;
  c->claimed = 0;
  c->happy = 0;
  c->sum.state = ST_RUNNING;
}

// A: w = sigma_j A u_j; partials of u_i . w (columns 0..j) and ||w||^2 (column j+1).
// Loads are issued in the order they are needed (stencil operands, then the basis values of
// the thread's row) before the launch tests whether it has work: the control block is read
// alongside, so the test costs no round trip of its own. A launch without work stores nothing.
template <int JM, class R, class Op>
__global__ __launch_bounds__(BS) void k_gmres_a(KArgs a, Op op, const double* __restrict__ V,
                                                size_t ldv, double* __restrict__ w, int j) {
  Ctl* c = a.ctl;
  const int state = c->sum.state, cj = c->j;
  const double sg = c->sigma[j];
  __shared__ typename Op::Lds L;
  __shared__ double red[NC_MAX * WAVES];
  __shared__ double red1[WAVES];
  const int nb = gridDim.x;
  const int lb = logical_block();
  const int row0 = lb * BS;
  const int nrows = tile_rows(a.n, row0);
  const int row = row0 + threadIdx.x;
  const bool mine = (int)threadIdx.x < nrows;
  const GatherX gx{V + (size_t)j * ldv};
  typename Op::template Pre<GatherX> pre{};
  if (nrows > 0) pre = op.load(row0, nrows, gx);
  const R rd(V, ldv, j + 1);
  double u[JM];
#pragma unroll
  for (int i = 0; i < JM; ++i) u[i] = (i <= j && mine) ? rd.load(i, row) : 0.0;
  const double y = nrows > 0 ? op.finish(pre, row0, nrows, gx, L) : 0.0;
  asm volatile("" ::: "memory");   // keeps the loads above ahead of the test below
  if (state != ST_RUNNING || cj != j) return;
  mark_work(c, a.pslot, a.mat_bytes + 8.0 * a.n * (j + 2));
  const double wr = mine ? sg * y : 0.0;
  if (mine) w[row] = wr;
#pragma unroll
  for (int i = 0; i < JM; ++i) u[i] *= wr;
  block_halving_partials<JM>(u, j + 1, a.partials, nb, lb, red);
  block_single_partial(wr * wr, a.partials, j + 1, nb, lb, red1);
}

// FA (j+2 workgroups): workgroup i <= j -> c1_i = sigma_i (u_i . w); workgroup j+1 -> ||A v_j||.
// The control words are read together with the partials (one memory round trip) and only the
// store depends on them.
__global__ __launch_bounds__(BS) void k_gmres_fin_a(Ctl* c, const double* partials, int nb,
                                                    int j) {
  __shared__ double lds[WAVES];
  const int col = blockIdx.x;
  const int state = c->sum.state, cj = c->j;
  const double sg = c->sigma[col];
  const double s = column_sum(partials + (size_t)col * nb, nb, lds);
  if (state != ST_RUNNING || cj != j || threadIdx.x != 0) return;
  if (col == j + 1) {
    c->wnorm_pre = sqrt(s);
  } else {
    const double c1 = sg * s;
    c->c1[col] = c1;
    c->d1[col] = c1 * sg;
  }
}

// B: w -= sum_i c1_i v_i (weights d1_i = c1_i sigma_i on the stored columns), then partials of
// u_i . w, sharing one read of the basis. Operands are requested before the work test, as in A.
template <int JM, class R>
__global__ __launch_bounds__(BS) void k_gmres_b(KArgs a, const double* __restrict__ V, size_t ldv,
                                                double* __restrict__ w, int j) {
  Ctl* c = a.ctl;
  const int state = c->sum.state, cj = c->j;
  __shared__ double red[NC_MAX * WAVES];
  const int t = threadIdx.x;
  const int nb = gridDim.x;
  const int lb = logical_block();
  const int row = lb * BS + t;
  const bool mine = row < a.n;
  double d[JM];   // uniform across the launch: scalar loads
#pragma unroll
  for (int i = 0; i < JM; ++i) d[i] = c->d1[i];
  const R rd(V, ldv, j + 1);
  double u[JM];
#pragma unroll
  for (int i = 0; i < JM; ++i) u[i] = (i <= j && mine) ? rd.load(i, row) : 0.0;
  double wr = mine ? w[row] : 0.0;
  asm volatile("" ::: "memory");
  if (state != ST_RUNNING || cj != j) return;
  mark_work(c, a.pslot, 8.0 * a.n * (j + 3));
#pragma unroll
  for (int i = 0; i < JM; ++i)
    if (i <= j) wr = fma(-d[i], u[i], wr);
  if (mine) w[row] = wr;
#pragma unroll
  for (int i = 0; i < JM; ++i) u[i] *= wr;
  block_halving_partials<JM>(u, j + 1, a.partials, nb, lb, red);
}

// FB (j+1 workgroups): c2_i = sigma_i (u_i . w).
__global__ __launch_bounds__(BS) void k_gmres_fin_b(Ctl* c, const double* partials, int nb,
                                                    int j) {
  __shared__ double lds[WAVES];
  const int col = blockIdx.x;
  const int state = c->sum.state, cj = c->j;
  const double sg = c->sigma[col];
  const double s = column_sum(partials + (size_t)col * nb, nb, lds);
  if (state != ST_RUNNING || cj != j || threadIdx.x != 0) return;
  const double c2 = sg * s;
  c->c2[col] = c2;
  c->d2[col] = c2 * sg;
}

// C: w -= sum_i c2_i v_i (weights d2_i = c2_i sigma_i), u_{j+1} = w, partial ||w||^2.
// Operands are requested before the work test, as in A.
template <int JM, class R>
__global__ __launch_bounds__(BS) void k_gmres_c(KArgs a, double* __restrict__ V, size_t ldv,
                                                const double* __restrict__ w, int j) {
  Ctl* c = a.ctl;
  const int state = c->sum.state, cj = c->j;
  __shared__ double red[WAVES];
  const int t = threadIdx.x;
  const int nb = gridDim.x;
  const int lb = logical_block();
  const int row = lb * BS + t;
  const bool mine = row < a.n;
  double d[JM];   // uniform across the launch: scalar loads
#pragma unroll
  for (int i = 0; i < JM; ++i) d[i] = c->d2[i];
  const R rd(V, ldv, j + 1);
  double u[JM];
#pragma unroll
  for (int i = 0; i < JM; ++i) u[i] = (i <= j && mine) ? rd.load(i, row) : 0.0;
  double wr = mine ? w[row] : 0.0;
  asm volatile("" ::: "memory");
  if (state != ST_RUNNING || cj != j) return;
  mark_work(c, a.pslot, 8.0 * a.n * (j + 3));
#pragma unroll
  for (int i = 0; i < JM; ++i)
    if (i <= j) wr = fma(-d[i], u[i], wr);
  if (mine) V[(size_t)(j + 1) * ldv + row] = wr;
  block_single_partial(wr * wr, a.partials, 0, nb, lb, red);
}

// FC (1 workgroup): Hessenberg column, Givens rotations, residual estimate; at the end of a
// cycle the k x k triangular solve H y = g (y stored pre-multiplied by sigma). Every control
// word the launch needs is requested before the first wait; the old rotations are applied in
// registers by one thread.
__global__ __launch_bounds__(BS) void k_gmres_fin_c(Ctl* c, const double* partials, int nb,
                                                    int j) {
  __shared__ double lds[WAVES];
  __shared__ double s_h[MMAX + 2];
  __shared__ double s_cs[MMAX], s_sn[MMAX];
  __shared__ int s_end, s_k;
  constexpr int LDH = MMAX + 1;
  const int t = threadIdx.x;
  const int state = c->sum.state, cj = c->j;
  const int iters = c->sum.iters, maxit = c->maxit, m = c->m;
  const double eps_b = c->eps_b, wpre = c->wnorm_pre, gj = c->g[j];
  const double ratio = c->ratio, ref = c->ref, tol = c->tol;
  if (t <= j) {
    s_h[t] = c->c1[t] + c->c2[t];
    s_cs[t] = c->cs[t];
    s_sn[t] = c->sn[t];
  }
  const double nrm2 = column_sum(partials, nb, lds);   // also orders the LDS writes above
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

// X: x += sum_{l<k} y_l v_l (y already carries sigma).
template <class R>
__global__ __launch_bounds__(BS) void k_gmres_x(KArgs a, const double* __restrict__ V, size_t ldv,
                                                double* __restrict__ x) {
  Ctl* c = a.ctl;
  if (c->sum.state != ST_CYCLE_END) return;
  __shared__ double s_y[MMAX];
  const int k = c->k;
  mark_work(c, a.pslot, 8.0 * a.n * (k + 2));
  const int t = threadIdx.x;
  if (t < k) s_y[t] = c->y[t];
  __syncthreads();
  const int row = logical_block() * BS + t;
  if (row >= a.n) return;
  const R rd(V, ldv, k > 0 ? k : 1);
  double acc = 0.0;
  for (int l = 0; l < k; ++l) acc = fma(s_y[l], rd.load(l, row), acc);
  x[row] = x[row] + acc;
}

// Arnoldi entry point: u_0 = r0, partial ||r0||^2.
__global__ __launch_bounds__(BS) void k_arnoldi_start(KArgs a, const double* __restrict__ r0,
                                                      double* __restrict__ u0, const int* flags) {
  Ctl* c = a.ctl;
  if (c->sum.state != ST_INIT || flags[0]) return;
  __shared__ double red[WAVES];
  const int nb = gridDim.x;
  const int lb = logical_block();
  const int row = lb * BS + threadIdx.x;
  double v = 0.0;
  if (row < a.n) {
    const double r = r0[row];
    u0[row] = r;
    v = r * r;
  }
  block_single_partial(v, a.partials, 0, nb, lb, red);
}

__global__ __launch_bounds__(BS) void k_arnoldi_fin_start(Ctl* c, const double* partials, int nb,
                                                          const int* flags) {
  if (c->sum.state != ST_INIT) return;
  if (flags[0]) {
    if (threadIdx.x == 0) {
      c->sum.state = ST_DONE;
      c->sum.status = -1;
    }
    return;
  }
  __shared__ double lds[WAVES];
  const double s = column_sum(partials, nb, lds);
  if (threadIdx.x != 0) return;
  const double nr = sqrt(s);
  if (!(nr > 0.0) || !isfinite(nr)) {
    c->sum.state = ST_DONE;
    c->sum.status = -2;
    return;
  }
  c->ref = 1.0;
  c->ratio = 1.0;
  c->sigma[0] = 1.0 / nr;
  c->g[0] = nr;
  for (int i = 1; i <= c->m; ++i) c->g[i] = 0.0;
  c->j = 0;
  c->sum.state = ST_RUNNING;
}

// Arnoldi entry point: normalise the stored columns in place and export H.
__global__ __launch_bounds__(BS) void k_arnoldi_finish(KArgs a, double* __restrict__ V, size_t ldv,
                                                       double* __restrict__ Hout, int m) {
  Ctl* c = a.ctl;
  if (c->sum.state != ST_CYCLE_END) return;
  const int k = c->k;
  const int cols = k + (c->happy ? 0 : 1);
  const int64_t total = (int64_t)a.n * cols;
  for (int64_t idx = (int64_t)blockIdx.x * BS + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * BS) {
    const int col = (int)(idx / a.n);
    const int row = (int)(idx % a.n);
    V[(size_t)col * ldv + row] *= c->sigma[col];
  }
  if (blockIdx.x == 0) {
    constexpr int LDH = MMAX + 1;
    for (int idx = threadIdx.x; idx < (m + 1) * m; idx += BS) {
      const int col = idx / (m + 1), row = idx % (m + 1);
      Hout[idx] = (col < k && row <= col + 1) ? c->Hraw[(size_t)col * LDH + row] : 0.0;
    }
  }
}

__global__ __launch_bounds__(64) void k_arnoldi_done(Ctl* c) {
  if (threadIdx.x == 0 && c->sum.state == ST_CYCLE_END) {
    c->sum.steps = c->k;
    c->sum.status = S_CONVERGED;
    c->sum.state = ST_DONE;
  }
}

// ---------------------------------------------------------------------------------------
// Host drivers
// ---------------------------------------------------------------------------------------
static int pick_jm(int cols) { return cols <= 8 ? 8 : cols <= 16 ? 16 : cols <= 32 ? 32 : 64; }

template <class R, class Op>
static hipError_t launch_step(const KArgs& ka, const Op& op, int nb, double* V, size_t ldv,
                              double* w, int j, hipStream_t s) {
  const int jm = pick_jm(j + 1);
  dim3 grid(nb), block(BS);
  KArgs kx = ka;
#define GSK_TIMED(CLS, LAUNCH)           \
  kx.pslot = probe_slot(CLS);            \
  if (kx.pslot >= 0) probe_begin(s);     \
  LAUNCH;                                \
  if (kx.pslot >= 0) probe_end(s, kx.pslot);
#define GSK_STEP(JMV)                                                                          \
  GSK_TIMED(KC_GMRES_A,                                                                        \
            hipLaunchKernelGGL((k_gmres_a<JMV, R, Op>), grid, block, 0, s, kx, op, V, ldv, w, j)) \
  hipLaunchKernelGGL(k_gmres_fin_a, dim3(j + 2), block, 0, s, ka.ctl, ka.partials, nb, j);     \
  GSK_TIMED(KC_GMRES_B,                                                                        \
            hipLaunchKernelGGL((k_gmres_b<JMV, R>), grid, block, 0, s, kx, V, ldv, w, j))      \
  hipLaunchKernelGGL(k_gmres_fin_b, dim3(j + 1), block, 0, s, ka.ctl, ka.partials, nb, j);     \
  GSK_TIMED(KC_GMRES_C,                                                                        \
            hipLaunchKernelGGL((k_gmres_c<JMV, R>), grid, block, 0, s, kx, V, ldv, w, j))      \
  hipLaunchKernelGGL(k_gmres_fin_c, dim3(1), block, 0, s, ka.ctl, ka.partials, nb, j);
  switch (jm) {
    case 8: GSK_STEP(8) break;
    case 16: GSK_STEP(16) break;
    case 32: GSK_STEP(32) break;
    default: GSK_STEP(64) break;
  }
#undef GSK_STEP
#undef GSK_TIMED
  return hipGetLastError();
}

template <class Op>
static void launch_residual(const KArgs& ka, const Op& op, int nb, const double* b,
                            const double* x, const double* W, double* u0, const int* flags,
                            hipStream_t s) {
  KArgs kx = ka;
  kx.pslot = probe_slot(KC_RESIDUAL);
  if (kx.pslot >= 0) probe_begin(s);
  hipLaunchKernelGGL(k_gmres_residual<Op>, dim3(nb), dim3(BS), 0, s, kx, op, b, x, W, u0, flags);
  if (kx.pslot >= 0) probe_end(s, kx.pslot);
  hipLaunchKernelGGL(k_gmres_fin_residual, dim3(1), dim3(BS), 0, s, ka.ctl,
                     (const double*)ka.partials, nb, W ? 1 : 0, flags);
}

static SolveResult fail(int code) {
  SolveResult r;
  r.code = code;
  r.sum = Summary{};
  return r;
}

template <class R, class Op>
static SolveResult gmres_run(const Mat& A, const Op& op, const double* b, double* x, int m,
                             const SolveParams& prm, void* ws, hipStream_t s) {
  Workspace W = carve(ws, A.n);
  const Geom g = make_geom(A.n);
  const size_t ldv = vec_ld(A.n);
  double* V = W.vecs;
  double* w = V + (size_t)(m + 1) * ldv;
  KArgs ka{A.n, g.rpb, W.ctl, W.partials, A.bytes(), -1};
  dim3 grid(g.nb), block(BS);
  if (launch_clear_flags(W.flags, s) != hipSuccess) return fail(-5);
  if (A.kind == MAT_CSR && launch_validate(A.csr, W.flags, s) != hipSuccess) return fail(-5);
  hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(64), 0, s, W.ctl, prm.maxit, m, prm.tol, prm.eps_b,
                     prm.weights ? 1 : 0);
  probe_solve_begin();
  launch_residual(ka, op, g.nb, b, x, prm.weights, V, W.flags, s);
  if (hipGetLastError() != hipSuccess) return fail(-5);

  Summary* hs = pinned_summaries();
  if (!hs) return fail(-5);
  hipEvent_t ev[2];
  if (hipEventCreateWithFlags(&ev[0], hipEventDisableTiming) != hipSuccess) return fail(-5);
  if (hipEventCreateWithFlags(&ev[1], hipEventDisableTiming) != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return fail(-5);
  }
  SolveResult res;
  res.code = 0;
  int slot = 0;
  bool pending = false, done = false;
  const long max_cycles = (long)prm.maxit + 8;
  Pacer pace{prm.tol, prm.maxit, m};
  if ((long)2 * m >= prm.maxit) pace.cautious = true;
  constexpr int kPiece = 10;   // steps per piece of a cycle in cautious mode
  auto steps = [&](int j0, int j1) {
    for (int j = j0; j < j1; ++j)
      if (launch_step<R>(ka, op, g.nb, V, ldv, w, j, s) != hipSuccess) return false;
    return true;
  };
  auto tail = [&]() {
    KArgs kx = ka;
    kx.pslot = probe_slot(KC_GMRES_X);
    if (kx.pslot >= 0) probe_begin(s);
    hipLaunchKernelGGL(k_gmres_x<R>, grid, block, 0, s, kx, (const double*)V, ldv, x);
    if (kx.pslot >= 0) probe_end(s, kx.pslot);
    launch_residual(ka, op, g.nb, b, x, prm.weights, V, W.flags, s);
    return hipGetLastError() == hipSuccess;
  };
  auto record = [&](int sl) {
    return hipMemcpyAsync(&hs[sl], &W.ctl->sum, sizeof(Summary), hipMemcpyDeviceToHost, s) ==
               hipSuccess &&
           hipEventRecord(ev[sl], s) == hipSuccess;
  };
  // Reads the status recorded in slot sl; false on a device error.
  auto check = [&](int sl) {
    if (hipEventSynchronize(ev[sl]) != hipSuccess) return false;
    if (hs[sl].state == ST_DONE) done = true;
    else pace.update(hs[sl].iters, hs[sl].relres_true);
    return true;
  };
  for (long cyc = 0; cyc <= max_cycles && !done; ++cyc) {
    if (!pace.cautious) {
      // Enqueue the whole cycle, then read the previous cycle's status while it runs.
      if (!steps(0, m) || !tail() || !record(slot)) { res.code = -5; break; }
      if (pending && !check(slot ^ 1)) { res.code = -5; break; }
      pending = true;
      slot ^= 1;
      continue;
    }
    if (pending) {   // first wait for the cycle still in flight
      if (!check(slot ^ 1)) { res.code = -5; break; }
      pending = false;
      if (done) break;
    }
    bool ok = true;
    for (int j0 = 0; j0 < m && ok; j0 += kPiece) {
      const int j1 = j0 + kPiece < m ? j0 + kPiece : m;
      ok = steps(j0, j1);
      if (!ok || j1 == m) break;
      // stop enqueueing this cycle once it has ended (convergence claimed, breakdown, cap)
      ok = record(slot) && hipEventSynchronize(ev[slot]) == hipSuccess;
      if (ok && hs[slot].state != ST_RUNNING) break;
    }
    if (!ok || !tail() || !record(slot) || !check(slot)) { res.code = -5; break; }
    slot ^= 1;
  }
  if (hipStreamSynchronize(s) != hipSuccess && res.code == 0) res.code = -5;
  if (res.code == 0) probe_collect(&W.ctl->probe, s);
  if (res.code == 0) {
    res.sum = hs[slot ^ 1];   // the most recent copy (state no longer changes once done)
    if (res.sum.state != ST_DONE) res.code = -5;
    else if (res.sum.status < 0) res.code = -1;
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  return res;
}

template <class R, class Op>
static SolveResult arnoldi_impl(const Mat& A, const Op& op, const double* r0, int m, double* V,
                                int64_t ldv, double* H, void* ws, double eps_b, hipStream_t s) {
  Workspace W = carve(ws, A.n);
  const Geom g = make_geom(A.n);
  double* w = W.vecs;
  KArgs ka{A.n, g.rpb, W.ctl, W.partials, A.bytes(), -1};
  dim3 grid(g.nb), block(BS);
  if (launch_clear_flags(W.flags, s) != hipSuccess) return fail(-5);
  if (A.kind == MAT_CSR && launch_validate(A.csr, W.flags, s) != hipSuccess) return fail(-5);
  // tol < 0: the estimate never ends the cycle; maxit = m steps.
  hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(64), 0, s, W.ctl, m, m, -1.0, eps_b, 0);
  probe_solve_begin();
  hipLaunchKernelGGL(k_arnoldi_start, grid, block, 0, s, ka, r0, V, (const int*)W.flags);
  hipLaunchKernelGGL(k_arnoldi_fin_start, dim3(1), block, 0, s, W.ctl,
                     (const double*)W.partials, g.nb, (const int*)W.flags);
  for (int j = 0; j < m; ++j)
    if (launch_step<R>(ka, op, g.nb, V, (size_t)ldv, w, j, s) != hipSuccess) return fail(-5);
  const int fin_blocks = 1024;
  hipLaunchKernelGGL(k_arnoldi_finish, dim3(fin_blocks), block, 0, s, ka, V, (size_t)ldv, H, m);
  hipLaunchKernelGGL(k_arnoldi_done, dim3(1), dim3(64), 0, s, W.ctl);
  if (hipGetLastError() != hipSuccess) return fail(-5);
  Summary* hs = pinned_summaries();
  if (!hs) return fail(-5);
  if (hipMemcpyAsync(&hs[0], &W.ctl->sum, sizeof(Summary), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(-5);
  probe_collect(&W.ctl->probe, s);
  SolveResult res;
  res.code = 0;
  res.sum = hs[0];
  if (res.sum.state != ST_DONE) res.code = -5;
  else if (res.sum.status < 0) res.code = -1;
  return res;
}

template <class Op>
static SolveResult gmres_dispatch(const Mat& A, const Op& op, const double* b, double* x, int m,
                                  const SolveParams& prm, void* ws, hipStream_t s) {
  if (fits_buffer(vec_ld(A.n), m + 1))
    return gmres_run<ColumnReader>(A, op, b, x, m, prm, ws, s);
  return gmres_run<PointerReader>(A, op, b, x, m, prm, ws, s);
}

SolveResult gmres_solve(const Mat& A, const double* b, double* x, int m, const SolveParams& prm,
                        void* ws, hipStream_t s) {
  if (A.kind == MAT_STENCIL) return gmres_dispatch(A, A.stencil_op(), b, x, m, prm, ws, s);
  return gmres_dispatch(A, A.csr_op(), b, x, m, prm, ws, s);
}

template <class Op>
static SolveResult arnoldi_dispatch(const Mat& A, const Op& op, const double* r0, int m,
                                    double* V, int64_t ldv, double* H, void* ws, double eps_b,
                                    hipStream_t s) {
  if (fits_buffer((size_t)ldv, m + 1))
    return arnoldi_impl<ColumnReader>(A, op, r0, m, V, ldv, H, ws, eps_b, s);
  return arnoldi_impl<PointerReader>(A, op, r0, m, V, ldv, H, ws, eps_b, s);
}

SolveResult arnoldi_run(const Mat& A, const double* r0, int m, double* V, int64_t ldv, double* H,
                        void* ws, double eps_b, hipStream_t s) {
  if (A.kind == MAT_STENCIL) return arnoldi_dispatch(A, A.stencil_op(), r0, m, V, ldv, H, ws, eps_b, s);
  return arnoldi_dispatch(A, A.csr_op(), r0, m, V, ldv, H, ws, eps_b, s);
}

}  // namespace gsk
