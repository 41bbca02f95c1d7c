// The batch engine's GMRES(m) launches: restarted GMRES with CGS2 Arnoldi (section 2) for many
// independent systems at once, in FP64 or with FP32 Arnoldi cycles and FP64 restarts (the
// iterative refinement of gsk_gmres_mixed).
//
// Every workgroup of a streaming launch takes one entry of the engine's unit list (a unit of
// one system's rows, see batch.hpp) and runs the same workgroup body as the single solver
// (gmres_body.hpp) on that system's rows, control block and slice of the basis; a finalize
// launch has one workgroup per system slot (and per column where the single solver has one
// per column) and reduces that system's partials in the single solver's order. A system
// therefore returns bit for bit what gsk_gmres (or gsk_gmres_mixed) returns for it alone.
//
// A chunk is one restart cycle for every running system: systems start their cycles together
// at the chunk's start, so step j of the chunk is step j of every running cycle and its
// launches are instantiated for j like the single solver's. Around the m steps:
//   prepare (GS stage, FP32 copy) -> start (residual of newly admitted systems)
//   -> A_0, FA_0, B_0, FB_0, C_0, then for j >= 1: A_j, FC_{j-1} beside FA_j, B_j, FB_j, C_j
//   -> FC_{m-1} -> X (x += V y at the cycle's end) -> restart (true residual: convergence
//   test, next cycle) -> summaries (control block -> status array).
// As in the single solver, A_j runs before FC_{j-1} (A multiplies the stored column), so C
// keeps its partials in a column of its own (GArgs::ccol) that A does not write.
#include "batch.hpp"
#include "gmres_body.hpp"

namespace gsk {

// Calls body(unit, slot) for the list entry of this workgroup; workgroups past the end of the
// list return at once.
template <class Body>
__device__ inline void on_unit(const GArgs& a, Body body) {
  const int k = logical_block();
  if (k < *a.n_act) body(a.act[k], a.act[a.max_units + k]);
}

__global__ __launch_bounds__(64) void k_bg_init(Ctl* c, int maxit, int m, double tol,
                                                double eps_b, int has_w, int prepare) {
  if (threadIdx.x != 0) return;
  c->sum.state = prepare ? ST_SCALE : ST_INIT;
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
  c->bad = 0;
  c->tol = tol;
  c->eps_b = eps_b;
  c->ref = 0.0;
  c->ratio = 1.0;
  c->wnorm_pre[0] = c->wnorm_pre[1] = 0.0;
  c->last_rt = 0.0;
}

// Preparation: GS(p) of the systems that asked for it, and the FP32 copy of the matrix.
template <class T>
__global__ __launch_bounds__(BS) void k_bg_prepare(GArgs a) {
  constexpr int RV = rpt_of<T>();
  __shared__ GsLds L;
  on_unit(a, [&](int unit, int s) {
    const SysDesc d = a.sys[s];
    Ctl* c = a.ctl + s;
    if (c->sum.state != ST_SCALE || (c->bad & BAD_CSR)) return;
    const int u = unit - d.unit_off;
#pragma unroll
    for (int q = 0; q < RV; ++q) {
      const int lt = u * RV + q;
      if (lt >= d.ntiles) break;
      prepare_tile(d, lt, L, &c->bad);
      __syncthreads();
    }
  });
}

__global__ __launch_bounds__(64) void k_bg_fin_prepare(GArgs a) {
  const int s = blockIdx.x;
  if (threadIdx.x != 0 || a.sys[s].ntiles == 0) return;
  Ctl* c = a.ctl + s;
  if (c->sum.state == ST_SCALE) c->sum.state = ST_INIT;   // errors are reported by FR
}

// R: true residual into u_0 (the tiles of the unit in turn; partials per tile).
template <class T>
__global__ __launch_bounds__(BS) void k_bg_residual(GArgs a) {
  constexpr int RV = rpt_of<T>();
  __shared__ TileLds L;
  __shared__ double red[NC_MAX * WAVES];
  on_unit(a, [&](int unit, int s) {
    const SysDesc d = a.sys[s];
    Ctl* c = a.ctl + s;
    const int bad = c->bad;
    T* u0 = static_cast<T*>(a.V) + d.row_off;
    const int u = unit - d.unit_off;
#pragma unroll
    for (int q = 0; q < RV; ++q) {
      const int lt = u * RV + q;
      if (lt >= d.ntiles) break;
      if (q) __syncthreads();
      if (d.kind == MAT_STENCIL) {
        EmptyLds e;
        const StencilOp op{d.coef, d.n, d.nx, d.ny, d.nz, (size_t)d.n};
        gmres_residual_tile<StencilOp, T>(c, op, d.n, d.b, d.x, d.W, u0, bad, lt,
                                          a.partials + d.tile_off, a.pstride, -1, 0.0, e, red);
      } else {
        const CsrOp op{d.rp, d.ci, d.val};
        gmres_residual_tile<CsrOp, T>(c, op, d.n, d.b, d.x, d.W, u0, bad, lt,
                                      a.partials + d.tile_off, a.pstride, -1, 0.0, L, red);
      }
    }
  });
}

__global__ __launch_bounds__(BS) void k_bg_fin_residual(GArgs a) {
  const int s = blockIdx.x;
  const SysDesc d = a.sys[s];
  if (d.ntiles == 0) return;
  Ctl* c = a.ctl + s;
  gmres_fin_residual_body(c, a.partials + d.tile_off, d.ntiles, a.pstride, d.W ? 1 : 0,
                          a.mixed, bad_status(c->bad));
}

// The matrix of the Arnoldi products: the FP64 scaled matrix, or its FP32 copy.
template <class T>
__device__ inline const T* inner_coef(const SysDesc& d) {
  if constexpr (sizeof(T) == 4) return d.mat32;
  else return d.coef;
}
template <class T>
__device__ inline const T* inner_val(const SysDesc& d) {
  if constexpr (sizeof(T) == 4) return d.mat32;
  else return d.val;
}
template <class T>
__device__ inline size_t inner_ldp(const SysDesc& d) {
  if constexpr (sizeof(T) == 4) return d.ldp32;
  else return (size_t)d.n;
}

// A_j. A stencil product takes the unit's RV tiles at once (partials per unit); a CSR product
// stages one tile at a time through LDS (partials per tile), as in the single solver. jexp:
// the step counter of a running step (j, or j-1 when FC_{j-1} runs after A_j).
// NT: the engine's admitted working set streams from HBM (see launch_gmres_chunk); the basis
// and the coefficient planes are then loaded non-temporally, and FP64 stencil products gather
// through the LDS window of StencilWinOpT. The bits are the same either way.
template <int JM, class R, class T, bool NT>
__global__ __launch_bounds__(BS) void k_bg_a(GArgs a, int j, int jexp) {
  constexpr int RV = rpt_of<T>();
  constexpr bool kWindow = NT && RV == 1;
  union Lds {
    TileLds csr;
    typename StencilWinOpT<double, NT>::Lds win;
  };
  __shared__ Lds L;
  __shared__ double red[NC_MAX * WAVES];
  __shared__ double red1[WAVES];
  on_unit(a, [&](int unit, int s) {
    const SysDesc d = a.sys[s];
    Ctl* c = a.ctl + s;
    const T* V = static_cast<const T*>(a.V) + d.row_off;
    T* w = static_cast<T*>(a.w) + d.row_off;
    const T zero = (T)a.zero;
    const int u = unit - d.unit_off;
    if (d.kind == MAT_STENCIL) {
      if constexpr (kWindow) {
        if (d.nx <= kWinNx) {
          const StencilWinOpT<double, NT> op{inner_coef<T>(d), d.n, d.nx, d.ny, d.nz,
                                             inner_ldp<T>(d)};
          gmres_a_tile<JM, RV, R, StencilWinOpT<double, NT>, T>(
              c, op, d.n, V, a.ldv, w, j, jexp, u, a.partials + d.unit_off, a.pstride, zero,
              -1, 0.0, L.win, red, red1);
          return;
        }
      }
      EmptyLds e;
      const StencilOpT<T, NT> op{inner_coef<T>(d), d.n, d.nx, d.ny, d.nz, inner_ldp<T>(d)};
      gmres_a_tile<JM, RV, R, StencilOpT<T, NT>, T>(c, op, d.n, V, a.ldv, w, j, jexp, u,
                                                    a.partials + d.unit_off, a.pstride, zero,
                                                    -1, 0.0, e, red, red1);
    } else {
      const CsrOpT<T> op{d.rp, d.ci, inner_val<T>(d)};
#pragma unroll
      for (int q = 0; q < RV; ++q) {
        const int lt = u * RV + q;
        if (lt >= d.ntiles) break;
        if (q) __syncthreads();
        gmres_a_tile<JM, 1, R, CsrOpT<T>, T>(c, op, d.n, V, a.ldv, w, j, jexp, lt,
                                             a.partials + d.tile_off, a.pstride, zero, -1, 0.0,
                                             L.csr, red, red1);
      }
    }
  });
}

// FA_j: grid (slots, j + 2).
template <class T>
__global__ __launch_bounds__(BS) void k_bg_fin_a(GArgs a, int j) {
  constexpr int RV = rpt_of<T>();
  __shared__ double lds[WAVES];
  const int s = blockIdx.x, col = blockIdx.y;
  const SysDesc d = a.sys[s];
  if (d.ntiles == 0) return;
  const bool per_tile = RV == 1 || d.kind != MAT_STENCIL;
  const int off = per_tile ? d.tile_off : d.unit_off;
  const int count = per_tile ? d.ntiles : d.nunits;
  gmres_fin_a_body(a.ctl + s, a.partials + off + (size_t)col * a.pstride, count, j, col, lds);
}

// FC_{j-1} beside FA_j (j >= 1): grid (slots, j + 3); blockIdx.y 0 runs FC, 1 + col the FA
// column col (see gmres_fin_a_body for what the two may not share).
template <class T>
__global__ __launch_bounds__(BS) void k_bg_fin_ca(GArgs a, int j) {
  constexpr int RV = rpt_of<T>();
  const int s = blockIdx.x;
  const SysDesc d = a.sys[s];
  if (d.ntiles == 0) return;
  const double* pc = a.partials + (size_t)a.ccol * a.pstride + d.unit_off;
  if (blockIdx.y == 0) {
    gmres_fin_c_body(a.ctl + s, pc, d.nunits, j - 1);
    return;
  }
  __shared__ double lds[WAVES];
  const int col = blockIdx.y - 1;
  const bool per_tile = RV == 1 || d.kind != MAT_STENCIL;
  const int off = per_tile ? d.tile_off : d.unit_off;
  const int count = per_tile ? d.ntiles : d.nunits;
  gmres_fin_a_body<true>(a.ctl + s, a.partials + off + (size_t)col * a.pstride, count, j, col,
                         lds, pc, d.nunits);
}

template <int JM, class R, class T>
__global__ __launch_bounds__(BS) void k_bg_b(GArgs a, int j) {
  constexpr int RV = rpt_of<T>();
  __shared__ double red[NC_MAX * WAVES];
  on_unit(a, [&](int unit, int s) {
    const SysDesc d = a.sys[s];
    const T* V = static_cast<const T*>(a.V) + d.row_off;
    T* w = static_cast<T*>(a.w) + d.row_off;
    gmres_b_tile<JM, RV, R, T>(a.ctl + s, d.n, V, a.ldv, w, j, unit - d.unit_off,
                               a.partials + d.unit_off, a.pstride, (T)a.zero, -1, red);
  });
}

// FB_j: grid (slots, j + 1).
__global__ __launch_bounds__(BS) void k_bg_fin_b(GArgs a, int j) {
  __shared__ double lds[WAVES];
  const int s = blockIdx.x, col = blockIdx.y;
  const SysDesc d = a.sys[s];
  if (d.ntiles == 0) return;
  gmres_fin_b_body(a.ctl + s, a.partials + d.unit_off + (size_t)col * a.pstride, d.nunits, j,
                   col, lds);
}

template <int JM, class R, class T>
__global__ __launch_bounds__(BS) void k_bg_c(GArgs a, int j) {
  constexpr int RV = rpt_of<T>();
  __shared__ double red[WAVES];
  on_unit(a, [&](int unit, int s) {
    const SysDesc d = a.sys[s];
    T* V = static_cast<T*>(a.V) + d.row_off;
    const T* w = static_cast<const T*>(a.w) + d.row_off;
    gmres_c_tile<JM, RV, R, T>(a.ctl + s, d.n, V, a.ldv, w, j, unit - d.unit_off,
                               a.partials + (size_t)a.ccol * a.pstride + d.unit_off, a.pstride,
                               (T)a.zero, -1, red);
  });
}

// FC_j: one workgroup per slot.
__global__ __launch_bounds__(BS) void k_bg_fin_c(GArgs a, int j) {
  const int s = blockIdx.x;
  const SysDesc d = a.sys[s];
  if (d.ntiles == 0) return;
  gmres_fin_c_body(a.ctl + s, a.partials + (size_t)a.ccol * a.pstride + d.unit_off, d.nunits, j);
}

template <class R, class T>
__global__ __launch_bounds__(BS) void k_bg_x(GArgs a) {
  constexpr int RV = rpt_of<T>();
  __shared__ double s_y[MMAX];
  on_unit(a, [&](int unit, int s) {
    const SysDesc d = a.sys[s];
    const T* V = static_cast<const T*>(a.V) + d.row_off;
    gmres_x_tile<RV, R, T>(a.ctl + s, d.n, V, a.ldv, d.x, unit - d.unit_off, -1, s_y);
  });
}

__global__ __launch_bounds__(64) void k_bg_sums(GArgs a) {
  const int s = blockIdx.x;
  if (threadIdx.x == 0 && a.sys[s].ntiles > 0) a.sums[s] = a.ctl[s].sum;
}

static int pick_jm(int cols) { return cols <= 8 ? 8 : cols <= 16 ? 16 : cols <= 32 ? 32 : 64; }

template <class R, class T, bool NT>
static hipError_t gmres_chunk(const GArgs& a, int m, int grid, int max_sys, hipStream_t s) {
  const dim3 gt(grid), gs(max_sys), block(BS);
  hipLaunchKernelGGL(k_bg_prepare<T>, gt, block, 0, s, a);
  hipLaunchKernelGGL(k_bg_fin_prepare, gs, dim3(64), 0, s, a);
  hipLaunchKernelGGL(k_bg_residual<T>, gt, block, 0, s, a);
  hipLaunchKernelGGL(k_bg_fin_residual, gs, block, 0, s, a);
  for (int j = 0; j < m; ++j) {
#define GSK_BG_STEP(JMV)                                                                     \
  hipLaunchKernelGGL((k_bg_a<JMV, R, T, NT>), gt, block, 0, s, a, j, j > 0 ? j - 1 : 0);     \
  if (j > 0)                                                                                 \
    hipLaunchKernelGGL(k_bg_fin_ca<T>, dim3(max_sys, j + 3), block, 0, s, a, j);             \
  else                                                                                       \
    hipLaunchKernelGGL(k_bg_fin_a<T>, dim3(max_sys, j + 2), block, 0, s, a, j);              \
  hipLaunchKernelGGL((k_bg_b<JMV, R, T>), gt, block, 0, s, a, j);                            \
  hipLaunchKernelGGL(k_bg_fin_b, dim3(max_sys, j + 1), block, 0, s, a, j);                   \
  hipLaunchKernelGGL((k_bg_c<JMV, R, T>), gt, block, 0, s, a, j);
    switch (pick_jm(j + 1)) {
      case 8: GSK_BG_STEP(8) break;
      case 16: GSK_BG_STEP(16) break;
      case 32: GSK_BG_STEP(32) break;
      default: GSK_BG_STEP(64) break;
    }
#undef GSK_BG_STEP
  }
  hipLaunchKernelGGL(k_bg_fin_c, gs, block, 0, s, a, m - 1);
  hipLaunchKernelGGL((k_bg_x<R, T>), gt, block, 0, s, a);
  hipLaunchKernelGGL(k_bg_residual<T>, gt, block, 0, s, a);
  hipLaunchKernelGGL(k_bg_fin_residual, gs, block, 0, s, a);
  hipLaunchKernelGGL(k_bg_sums, gs, dim3(64), 0, s, a);
  return hipGetLastError();
}

template <bool NT>
static hipError_t gmres_chunk_nt(const GArgs& a, int m, int grid, int max_sys, bool column,
                                 hipStream_t s) {
  if (a.mixed) {
    if (column)
      return gmres_chunk<ColumnReaderT<float, NT>, float, NT>(a, m, grid, max_sys, s);
    return gmres_chunk<PointerReaderT<float, NT>, float, NT>(a, m, grid, max_sys, s);
  }
  if (column) return gmres_chunk<ColumnReaderT<double, NT>, double, NT>(a, m, grid, max_sys, s);
  return gmres_chunk<PointerReaderT<double, NT>, double, NT>(a, m, grid, max_sys, s);
}

hipError_t launch_gmres_chunk(const GArgs& a, int m, int grid, int max_sys, bool column,
                              bool nt, hipStream_t s) {
  return nt ? gmres_chunk_nt<true>(a, m, grid, max_sys, column, s)
            : gmres_chunk_nt<false>(a, m, grid, max_sys, column, s);
}

hipError_t launch_gmres_init(Ctl* c, int maxit, int m, double tol, double eps_b, int has_w,
                             int prepare, hipStream_t s) {
  hipLaunchKernelGGL(k_bg_init, dim3(1), dim3(64), 0, s, c, maxit, m, tol, eps_b, has_w,
                     prepare);
  return hipGetLastError();
}

}  // namespace gsk
