// Restarted GMRES(m) with double classical Gram-Schmidt (CGS2) Arnoldi, and the bare
// Arnoldi process, on the device.
//
// Section 2 of the paper: restarted GMRES whose Arnoldi step orthogonalises with a double
// classical Gram-Schmidt pass. One Arnoldi step j (basis columns u_0..u_j stored unnormalised
// with scale factors sigma_i, so v_i = sigma_i u_i) is three streaming launches and the small
// finalize launches that reduce their per-workgroup partials:
//
//   A  w = A u_j (tile product), partial V_j^T w, ||w||^2           reads A, V_j; writes w
//      FA: c1_i = sigma_i (u_i . w), ||w||                          (j+2 workgroups)
//   B  w -= V_j c1, partial V_j^T w                                  reads V_j, w; writes w
//      FB: c2_i                                                     (j+1 workgroups)
//   C  u_{j+1} = sigma_j (w - V_j c2), partial ||u_{j+1}||^2          reads V_j, w; writes u
//      FC: h_{.,j} = sigma_j (c1 + c2), h_{j+1,j} = ||u_{j+1}||, Givens rotations, residual
//          estimate, and at the end of a cycle the triangular solve for y   (1 workgroup)
//
// The basis is read three times per step instead of four: the update of pass 1 and the dot
// products of pass 2 share one read, with the basis values held in registers. The division
// v_{j+1} = w / h_{j+1,j} is never materialised: sigma_{j+1} = 1/h_{j+1,j} is folded into the
// coefficients of later passes. A multiplies the stored column u_j, not v_j, so that it needs
// nothing from FC of step j-1; the factor sigma_j is applied by C and FC. That lets one launch
// run FC of step j-1 (workgroup 0) beside FA of step j (the other workgroups), after A of
// step j: five launches per step instead of six. A then runs before it is known whether step
// j-1 ended the cycle; if it did, the cycle's remaining launches find the cycle ended and
// store nothing, and the sums of that step are never read. The first step of each enqueued
// run of steps uses the plain FA, the last one the plain FC. At the end of a cycle X adds
// V_k y to x and R (+ FR) recomputes the true residual r = b - A x, which either ends the
// solve or starts the next cycle with u_0 = r.
//
// Every launch checks the device-resident state and stores nothing if the solve has moved on
// (the merged launch's FA workgroups excepted, see gmres_fin_a_body), so a whole cycle can be
// enqueued blindly; the host reads a small summary once per cycle.
//
// Storage precision. The kernels are templated on T, the type the basis and w are stored in,
// and on the operator of the inner product. With T = double and the caller's matrix this is
// the FP64 solver. With T = float and an FP32 copy of the matrix it is the mixed-precision
// solver (gsk_gmres_mixed): each cycle's Arnoldi process reads and writes FP32 data while all
// arithmetic, the Hessenberg matrix, the rotations and y stay FP64, and every restart
// computes the true residual r = b - A x and updates x in FP64 with the caller's matrix. That
// is iterative refinement with one GMRES(m) cycle per correction. Every value a kernel uses
// after storing it is the stored (rounded) value, so the Arnoldi relation holds for the data
// in memory.
#include "gmres_body.hpp"
#include "gsk_host.hpp"

namespace gsk {

struct KArgs {
  int n;
  int rpb;
  Ctl* ctl;
  double* partials;
  double mat_bytes;     // algorithmic bytes of one read of A (CSR: 12 nnz + 4 (n+1))
  int pslot;            // measurement slot of this launch, or -1
  double inner_bytes;   // bytes of one read of the matrix the Arnoldi product uses
  // 0.0, passed at run time: the value of a basis entry that is not loaded. As a constant
  // the compiler would move the later FP32 -> FP64 widening into the conditional load's
  // block, which makes each load wait for its data before the next one is issued.
  double zero;
  // C's partials, apart from A's columns: A of step j runs before FC of step j-1 reads them.
  double* cpartials;
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
  c->sum.fp64_from = 0;
  c->sum.pad0 = 0;
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
  c->wnorm_pre[0] = c->wnorm_pre[1] = 0.0;
  c->last_rt = 0.0;
}

// The workgroup bodies of the kernels below are in gmres_body.hpp (shared with the batch
// engine). Here each workgroup takes the rows of its XCD-aware index (one tile of BS rows per
// workgroup, or RPT tiles), and the partials have one entry per workgroup of the grid.

// R: r = b - A x (FP64, the caller's matrix) into u_0 stored as T; partials ||r||^2
// (column 0), ||W r||^2 (column 1) and ||u_0||^2 of the stored values (column 2).
template <class Op, class T>
__global__ __launch_bounds__(BS) void k_gmres_residual(KArgs a, Op op, const double* __restrict__ b,
                                                       const double* __restrict__ x,
                                                       const double* __restrict__ W,
                                                       T* __restrict__ u0, const int* flags) {
  __shared__ typename Op::Lds L;
  __shared__ double red[NC_MAX * WAVES];
  gmres_residual_tile<Op, T>(a.ctl, op, a.n, b, x, W, u0, flags[0], logical_block(), a.partials,
                             gridDim.x, a.pslot, a.mat_bytes, L, red);
}

// FR: convergence / restart decision after the true residual (see file comment).
// In the mixed-precision solver (mixed = 1) an FP32 cycle may claim convergence that the
// FP64 residual does not confirm simply because FP32 data cannot resolve the last digits; such
// a cycle still counts as progress when it halved the true residual, and only claims without
// progress count towards STAGNATED.
__global__ __launch_bounds__(BS) void k_gmres_fin_residual(Ctl* c, const double* partials,
                                                           int nb, int has_w, int mixed,
                                                           const int* flags) {
  gmres_fin_residual_body(c, partials, nb, nb, has_w, mixed, flags[0] ? -1 : 0);
}

// A: w = A u_j; partials of u_i . w (columns 0..j) and ||w||^2 (column j+1). jexp: the step
// counter the step runs at (j, or j-1 when the merged launch follows).
template <int JM, int RPT, class R, class Op, class T>
__global__ __launch_bounds__(BS) void k_gmres_a(KArgs a, Op op, const T* __restrict__ V,
                                                size_t ldv, T* __restrict__ w, int j, int jexp) {
  __shared__ typename Op::Lds L;
  __shared__ double red[NC_MAX * WAVES];
  __shared__ double red1[WAVES];
  gmres_a_tile<JM, RPT, R, Op, T>(a.ctl, op, a.n, V, ldv, w, j, jexp, logical_block(),
                                  a.partials, gridDim.x, (T)a.zero, a.pslot, a.inner_bytes, L,
                                  red, red1);
}

// FA (j+2 workgroups): workgroup i <= j -> c1_i = sigma_i (u_i . w); workgroup j+1 -> ||w||.
// BIG: partial sums of more than SUM_BATCH * BS tiles, with larger batches of loads (the same
// order of additions).
template <bool BIG>
__global__ __launch_bounds__(BS) void k_gmres_fin_a(Ctl* c, const double* partials, int nb,
                                                    int j) {
  __shared__ double lds[WAVES];
  const int col = blockIdx.x;
  gmres_fin_a_body<false, BIG ? sum_batch<1>() : SUM_BATCH>(c, partials + (size_t)col * nb,
                                                            nb, j, col, lds);
}

// FC of step j-1 and FA of step j (j >= 1) in one launch of j+3 workgroups: workgroup 0 runs
// FC on C's nbc partials, workgroup 1+i the FA column i on A's nba partials.
template <bool BIG>
__global__ __launch_bounds__(BS) void k_gmres_fin_ca(Ctl* c, const double* pa, int nba,
                                                     const double* pc, int nbc, int j) {
  constexpr int SB = BIG ? sum_batch<1>() : SUM_BATCH;
  if (blockIdx.x == 0) {
    gmres_fin_c_body<SB>(c, pc, nbc, j - 1);
    return;
  }
  __shared__ double lds[WAVES];
  const int col = blockIdx.x - 1;
  gmres_fin_a_body<true, SB>(c, pa + (size_t)col * nba, nba, j, col, lds, pc, nbc);
}

// B: w -= sum_i c1_i v_i, then partials of u_i . w, sharing one read of the basis.
template <int JM, int RPT, class R, class T>
__global__ __launch_bounds__(BS) void k_gmres_b(KArgs a, const T* __restrict__ V, size_t ldv,
                                                T* __restrict__ w, int j) {
  __shared__ double red[NC_MAX * WAVES];
  gmres_b_tile<JM, RPT, R, T>(a.ctl, a.n, V, ldv, w, j, logical_block(), a.partials, gridDim.x,
                              (T)a.zero, a.pslot, red);
}

// FB (j+1 workgroups): c2_i = sigma_i (u_i . w).
template <bool BIG>
__global__ __launch_bounds__(BS) void k_gmres_fin_b(Ctl* c, const double* partials, int nb,
                                                    int j) {
  __shared__ double lds[WAVES];
  const int col = blockIdx.x;
  gmres_fin_b_body<BIG ? sum_batch<1>() : SUM_BATCH>(c, partials + (size_t)col * nb, nb, j,
                                                     col, lds);
}

// C: u_{j+1} = sigma_j (w - sum_i c2_i v_i), partial ||u_{j+1}||^2 (into cpartials).
template <int JM, int RPT, class R, class T>
__global__ __launch_bounds__(BS) void k_gmres_c(KArgs a, T* __restrict__ V, size_t ldv,
                                                const T* __restrict__ w, int j) {
  __shared__ double red[WAVES];
  gmres_c_tile<JM, RPT, R, T>(a.ctl, a.n, V, ldv, w, j, logical_block(), a.cpartials,
                              gridDim.x, (T)a.zero, a.pslot, red);
}

// FC (1 workgroup): Hessenberg column, Givens rotations, residual estimate; at the end of a
// cycle the triangular solve for y.
template <bool BIG>
__global__ __launch_bounds__(BS) void k_gmres_fin_c(Ctl* c, const double* partials, int nb,
                                                    int j) {
  gmres_fin_c_body<BIG ? sum_batch<1>() : SUM_BATCH>(c, partials, nb, j);
}

// X: x += sum_{l<k} y_l v_l (y already carries sigma).
template <int RPT, class R, class T>
__global__ __launch_bounds__(BS) void k_gmres_x(KArgs a, const T* __restrict__ V, size_t ldv,
                                                double* __restrict__ x) {
  __shared__ double s_y[MMAX];
  gmres_x_tile<RPT, R, T>(a.ctl, a.n, V, ldv, x, logical_block(), a.pslot, s_y);
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

// Step j. merged: FC of step j-1 has not run yet (it runs in the launch after A); else FC of
// every earlier step has run. FC of step j itself is left to the next step or to
// launch_fin_c.
template <class R, class Op, class T>
static hipError_t launch_step(const KArgs& ka, const Op& op, int n, T* V, size_t ldv, T* w,
                              int j, bool merged, hipStream_t s) {
  constexpr int RV = rpt_of<T>();                  // B, C: rows per thread
  constexpr int RA = Op::kRowwise ? RV : 1;        // A
  const int ga = grid_for(n, RA), gv = grid_for(n, RV);
  const int jm = pick_jm(j + 1);
  const bool big = (ga > gv ? ga : gv) > SUM_BATCH * BS;   // finalize with larger batches
  dim3 block(BS);
  KArgs kx = ka;
#define GSK_STEP(JMV)                                                                          \
  kx.pslot = probe_slot(KC_GMRES_A);                                                           \
  launch_probed(k_gmres_a<JMV, RA, R, Op, T>, dim3(ga), s, kx.pslot, kx, op, (const T*)V, ldv, \
                w, j, merged ? j - 1 : j);                                                     \
  if (merged)                                                                                  \
    hipLaunchKernelGGL(big ? k_gmres_fin_ca<true> : k_gmres_fin_ca<false>, dim3(j + 3), block, \
                       0, s, ka.ctl, (const double*)ka.partials, ga,                           \
                       (const double*)ka.cpartials, gv, j);                                    \
  else                                                                                         \
    hipLaunchKernelGGL(big ? k_gmres_fin_a<true> : k_gmres_fin_a<false>, dim3(j + 2), block,   \
                       0, s, ka.ctl, ka.partials, ga, j);                                      \
  kx.pslot = probe_slot(KC_GMRES_B);                                                           \
  launch_probed(k_gmres_b<JMV, RV, R, T>, dim3(gv), s, kx.pslot, kx, (const T*)V, ldv, w, j);  \
  hipLaunchKernelGGL(big ? k_gmres_fin_b<true> : k_gmres_fin_b<false>, dim3(j + 1), block, 0, \
                     s, ka.ctl, ka.partials, gv, j);                                           \
  kx.pslot = probe_slot(KC_GMRES_C);                                                           \
  launch_probed(k_gmres_c<JMV, RV, R, T>, dim3(gv), s, kx.pslot, kx, V, ldv, (const T*)w, j);
  switch (jm) {
    case 8: GSK_STEP(8) break;
    case 16: GSK_STEP(16) break;
    case 32: GSK_STEP(32) break;
    default: GSK_STEP(64) break;
  }
#undef GSK_STEP
  return hipGetLastError();
}

// The plain FC of step j (after the last step of an enqueued run of steps).
template <class T>
static hipError_t launch_fin_c(const KArgs& ka, int n, int j, hipStream_t s) {
  const int gv = grid_for(n, rpt_of<T>());
  hipLaunchKernelGGL(gv > SUM_BATCH * BS ? k_gmres_fin_c<true> : k_gmres_fin_c<false>, dim3(1),
                     dim3(BS), 0, s, ka.ctl, (const double*)ka.cpartials, gv, j);
  return hipGetLastError();
}

// Steps j0..j1-1 (j0 < j1): the first with the plain FA, the others with the merged launch,
// and the plain FC of step j1-1 last, so that no step is left unfinished.
template <class R, class Op, class T>
static hipError_t launch_steps(const KArgs& ka, const Op& op, int n, T* V, size_t ldv, T* w,
                               int j0, int j1, hipStream_t s) {
  for (int j = j0; j < j1; ++j) {
    const hipError_t e = launch_step<R>(ka, op, n, V, ldv, w, j, j > j0, s);
    if (e != hipSuccess) return e;
  }
  return launch_fin_c<T>(ka, n, j1 - 1, s);
}

template <class Op, class T>
static void launch_residual(const KArgs& ka, const Op& op, int nb, const double* b,
                            const double* x, const double* W, T* u0, const int* flags, int mixed,
                            hipStream_t s) {
  KArgs kx = ka;
  kx.pslot = probe_slot(KC_RESIDUAL);
  launch_probed(k_gmres_residual<Op, T>, dim3(nb), s, kx.pslot, kx, op, b, x, W, u0, flags);
  hipLaunchKernelGGL(k_gmres_fin_residual, dim3(1), dim3(BS), 0, s, ka.ctl,
                     (const double*)ka.partials, nb, W ? 1 : 0, mixed, flags);
}

// FP64 -> FP32 copy of matrix values (the mixed-precision solver's inner matrix): `segs`
// segments of `len` values, read with stride src_ld and written with stride dst_ld.
__global__ __launch_bounds__(BS) void k_to_f32(const double* __restrict__ src, size_t src_ld,
                                               float* __restrict__ dst, size_t dst_ld,
                                               int64_t len, int segs) {
  const int64_t total = len * segs;
  for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * BS) {
    const int64_t sg = i / len, k = i - sg * len;
    dst[sg * dst_ld + k] = (float)src[sg * src_ld + k];
  }
}

static SolveResult fail(int code) {
  SolveResult r;
  r.code = code;
  r.sum = Summary{};
  return r;
}

// Restarted GMRES(m): Op64 is the caller's FP64 matrix (true residuals), OpT the matrix the
// Arnoldi products use (the same one, or its FP32 copy), T the storage type of V (m+1 columns
// of ld values) and w. mixed selects the refinement form of the stagnation rule.
template <class R, class Op64, class OpT, class T>
static SolveResult gmres_run(const Mat& A, const Op64& op, const OpT& opT, double inner_bytes,
                             const double* b, double* x, int m, const SolveParams& prm,
                             void* ws, T* V, int mixed, hipStream_t s) {
  Workspace W = carve(ws, A.n);
  const Geom g = make_geom(A.n);
  const size_t ldv = vec_ld(A.n);
  T* w = V + (size_t)(m + 1) * ldv;
  KArgs ka{A.n, g.rpb, W.ctl, W.partials, A.bytes(), -1, inner_bytes, 0.0,
           W.partials + (size_t)(NC_MAX - 1) * g.nb};
  dim3 grid(g.nb);
  if (launch_clear_flags(W.flags, s) != hipSuccess) return fail(-5);
  if (A.kind == MAT_CSR && launch_validate(A.csr, W.flags, s) != hipSuccess) return fail(-5);
  hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(64), 0, s, W.ctl, prm.maxit, m, prm.tol, prm.eps_b,
                     prm.weights ? 1 : 0);
  probe_solve_begin();
  launch_residual(ka, op, g.nb, b, x, prm.weights, V, W.flags, mixed, s);
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
    return launch_steps<R>(ka, opT, A.n, V, ldv, w, j0, j1, s) == hipSuccess;
  };
  auto tail = [&]() {
    KArgs kx = ka;
    kx.pslot = probe_slot(KC_GMRES_X);
    launch_probed(k_gmres_x<rpt_of<T>(), R, T>, dim3(grid_for(A.n, rpt_of<T>())), s, kx.pslot,
                  kx, (const T*)V, ldv, x);
    launch_residual(ka, op, g.nb, b, x, prm.weights, V, W.flags, mixed, s);
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
  KArgs ka{A.n, g.rpb, W.ctl, W.partials, A.bytes(), -1, A.bytes(), 0.0,
           W.partials + (size_t)(NC_MAX - 1) * g.nb};
  dim3 grid(g.nb), block(BS);
  if (launch_clear_flags(W.flags, s) != hipSuccess) return fail(-5);
  if (A.kind == MAT_CSR && launch_validate(A.csr, W.flags, s) != hipSuccess) return fail(-5);
  // tol < 0: the estimate never ends the cycle; maxit = m steps.
  hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(64), 0, s, W.ctl, m, m, -1.0, eps_b, 0);
  probe_solve_begin();
  hipLaunchKernelGGL(k_arnoldi_start, grid, block, 0, s, ka, r0, V, (const int*)W.flags);
  hipLaunchKernelGGL(k_arnoldi_fin_start, dim3(1), block, 0, s, W.ctl,
                     (const double*)W.partials, g.nb, (const int*)W.flags);
  if (launch_steps<R>(ka, op, A.n, V, (size_t)ldv, w, 0, m, s) != hipSuccess) return fail(-5);
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

// Cache policy by working-set size. A cycle's working set (basis, w and the matrix the Arnoldi
// products read) that exceeds the last-level cache (256 MB of Infinity Cache on MI355X) is
// streamed from HBM once per launch whatever the policy; then the basis and the coefficient
// planes are loaded non-temporally, which keeps the caches for the gathered column's
// neighbours and the partials. Below that size the data stays cache-resident between launches
// and ordinary loads are faster. Results are the same bits either way.

static bool streams(const Mat& A, int m, size_t value_bytes, double inner_bytes) {
  return (double)(m + 2) * (double)vec_ld(A.n) * (double)value_bytes + inner_bytes >
         kStreamBytes;
}

template <bool NT, class Op, class OpT>
static SolveResult gmres_dispatch_nt(const Mat& A, const Op& op, const OpT& opT,
                                     const double* b, double* x, int m, const SolveParams& prm,
                                     void* ws, hipStream_t s) {
  double* V = carve(ws, A.n).vecs;
  if (fits_buffer<double>(vec_ld(A.n), m + 1))
    return gmres_run<ColumnReaderT<double, NT>>(A, op, opT, A.bytes(), b, x, m, prm, ws, V, 0,
                                                s);
  return gmres_run<PointerReaderT<double, NT>>(A, op, opT, A.bytes(), b, x, m, prm, ws, V, 0,
                                               s);
}

SolveResult gmres_solve(const Mat& A, const double* b, double* x, int m, const SolveParams& prm,
                        void* ws, hipStream_t s) {
  const bool nt = streams(A, m, sizeof(double), A.bytes());
  if (A.kind == MAT_STENCIL) {
    const StencilOp op = A.stencil_op();
    if (nt) {
      // a streamed working set: the Arnoldi product gathers through the LDS window (the same
      // bits as the plain stencil product)
      if (A.nx <= kWinNx) {
        const StencilWinOpT<double, true> opw{A.coef, A.n, A.nx, A.ny, A.nz, (size_t)A.n};
        return gmres_dispatch_nt<true>(A, op, opw, b, x, m, prm, ws, s);
      }
      const StencilOpT<double, true> opn{A.coef, A.n, A.nx, A.ny, A.nz, (size_t)A.n};
      return gmres_dispatch_nt<true>(A, op, opn, b, x, m, prm, ws, s);
    }
    return gmres_dispatch_nt<false>(A, op, op, b, x, m, prm, ws, s);
  }
  if (nt) return gmres_dispatch_nt<true>(A, A.csr_op(), A.csr_op(), b, x, m, prm, ws, s);
  return gmres_dispatch_nt<false>(A, A.csr_op(), A.csr_op(), b, x, m, prm, ws, s);
}

// Mixed precision: [head | FP32 copy of the matrix values | V (m+1 columns) | w], FP32.
// The FP32 planes are padded to vec_ld(n) values each, so every plane starts 256-byte aligned.
size_t mixed_matrix_floats(const Mat& A) {
  return A.kind == MAT_STENCIL ? (size_t)A.planes() * vec_ld(A.n) : (size_t)A.csr.nnz;
}

template <class Op64, class OpT>
static SolveResult gmres_mixed_dispatch(const Mat& A, const Op64& op, const OpT& opT,
                                        double inner_bytes, float* V, const double* b, double* x,
                                        int m, const SolveParams& prm, void* ws, hipStream_t s) {
  if (fits_buffer<float>(vec_ld(A.n), m + 1))
    return gmres_run<ColumnReaderT<float>>(A, op, opT, inner_bytes, b, x, m, prm, ws, V, 1, s);
  return gmres_run<PointerReaderT<float>>(A, op, opT, inner_bytes, b, x, m, prm, ws, V, 1, s);
}

SolveResult gmres_mixed_solve(const Mat& A, const double* b, double* x, int m,
                              const SolveParams& prm, void* ws, hipStream_t s) {
  char* base = reinterpret_cast<char*>(carve(ws, A.n).vecs);
  float* vals = reinterpret_cast<float*>(base);
  float* V = reinterpret_cast<float*>(base + align256(sizeof(float) * mixed_matrix_floats(A)));
  const bool st = A.kind == MAT_STENCIL;
  const int64_t len = st ? (int64_t)A.n : (int64_t)A.csr.nnz;
  const int segs = st ? A.planes() : 1;
  int64_t blocks = (len * segs + BS - 1) / BS;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)blocks), dim3(BS), 0, s,
                     st ? A.coef : A.csr.val, (size_t)len, vals, st ? vec_ld(A.n) : (size_t)len,
                     len, segs);
  if (hipGetLastError() != hipSuccess) return fail(-5);
  if (A.kind == MAT_STENCIL) {
    // FP32 planes beyond the cache are streamed non-temporally (the FP32 basis keeps ordinary
    // loads: measured faster for the mixed solver at 160^3)
    const double inner = 4.0 * A.planes() * A.n;
    if (streams(A, m, sizeof(float), inner)) {
      const StencilOpT<float, true> opT{vals, A.n, A.nx, A.ny, A.nz, vec_ld(A.n)};
      return gmres_mixed_dispatch(A, A.stencil_op(), opT, inner, V, b, x, m, prm, ws, s);
    }
    const StencilOpT<float> opT{vals, A.n, A.nx, A.ny, A.nz, vec_ld(A.n)};
    return gmres_mixed_dispatch(A, A.stencil_op(), opT, inner, V, b, x, m, prm, ws, s);
  }
  const CsrOpT<float> opT{A.csr.rp, A.csr.ci, vals};
  return gmres_mixed_dispatch(A, A.csr_op(), opT, 8.0 * A.csr.nnz + 4.0 * (A.n + 1.0), V, b, x,
                              m, prm, ws, s);
}

template <class Op>
static SolveResult arnoldi_dispatch(const Mat& A, const Op& op, const double* r0, int m,
                                    double* V, int64_t ldv, double* H, void* ws, double eps_b,
                                    hipStream_t s) {
  if (fits_buffer<double>((size_t)ldv, m + 1))
    return arnoldi_impl<ColumnReader>(A, op, r0, m, V, ldv, H, ws, eps_b, s);
  return arnoldi_impl<PointerReader>(A, op, r0, m, V, ldv, H, ws, eps_b, s);
}

SolveResult arnoldi_run(const Mat& A, const double* r0, int m, double* V, int64_t ldv, double* H,
                        void* ws, double eps_b, hipStream_t s) {
  if (A.kind == MAT_STENCIL) return arnoldi_dispatch(A, A.stencil_op(), r0, m, V, ldv, H, ws, eps_b, s);
  return arnoldi_dispatch(A, A.csr_op(), r0, m, V, ldv, H, ws, eps_b, s);
}

}  // namespace gsk
