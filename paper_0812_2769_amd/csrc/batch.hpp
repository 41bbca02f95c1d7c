// Shared by the batch engine's files (batch.hip: the engine and its Bi-CGSTAB kernels;
// batch_gmres.hip: its GMRES kernels).
#pragma once

#include "gsk_host.hpp"

namespace gsk {

// One admitted system. Its rows occupy tiles [tile_off, tile_off + ntiles) of the engine's
// row space (row_off = tile_off * BS); a workgroup of a streaming launch takes one unit of
// `units` consecutive tiles (1, or 2 for FP32 data), units [unit_off, unit_off + nunits).
// cls: the size class whose launches take the system (0 when the engine has one class).
struct SysDesc {
  int n, kind, nx, ny, nz, tile_off, ntiles, gs_p;
  int unit_off, nunits, cls;
  int64_t row_off;
  const int* rp;
  const int* ci;
  const double* val;      // CSR values the solve reads (the GS output with a GS stage)
  const double* coef;     // stencil planes the solve reads (likewise)
  const double* b;        // right-hand side the solve reads (likewise)
  double* x;
  const double* W;        // stop weights (written by the GS stage for p != 2)
  const double* gs_val;   // GS stage input: unscaled values or planes
  const double* gs_b;     // GS stage input: unscaled b
  const float* mat32;     // FP32 copy of the scaled matrix (mixed GMRES): planes or values
  size_t ldp32;           // plane stride of mat32 for a stencil matrix
};

// Per-system control block of a Bi-CGSTAB engine (the Bi-CGSTAB part of Ctl). target and
// last_rt serve the mixed-precision form: the run's stop level max(tol, delta * rt) and the
// relative true residual rt its run started from.
struct BCtl {
  Summary sum;
  int maxit, first, has_w, bad;
  int fp64;         // mixed engine: the system continues in FP64 (FP64 engine: unused)
  int run_start;    // mixed engine: iteration count at the start of the current float run
  double tol, eps_b, ref;
  double rho, rho_old, alpha, omega, beta, rh_norm;
  double target, last_rt;
};

// Bits of rejected system data: invalid CSR structure, zero row, non-finite data (GS stage).
enum : int { BAD_CSR = 1, BAD_ZERO = 2, BAD_NONFINITE = 4 };

__device__ inline int bad_status(int bad) {
  return bad == 0 ? 0 : (bad & BAD_CSR) ? -1 : (bad & BAD_ZERO) ? -2 : -3;
}

// Preparation of one tile (system-local index lt) of a system that asked for it: GS(p) into
// the system's outputs with the arithmetic of gsk_gs_scale (and, if it has one, the FP32 copy
// of the scaled values), or, without a GS stage, only the FP32 copy of its (already scaled)
// matrix. Zero rows and non-finite data set bits in *bad. All threads of the workgroup call.
__device__ inline void prepare_tile(const SysDesc& d, int lt, GsLds& L, int* bad) {
  const int row0 = lt * BS;
  const int nrows = min(BS, d.n - row0);
  const int t = threadIdx.x;
  float* m32 = const_cast<float*>(d.mat32);
  if (d.gs_p > 0) {
    bool zero = false, nonfinite = false;
    if (d.kind == MAT_STENCIL) {
      if (t < nrows)
        gs_stencil_row(d.gs_val, (size_t)d.n, d.n, d.nx, d.ny, d.nz, d.gs_b, d.gs_p, row0 + t,
                       const_cast<double*>(d.coef), const_cast<double*>(d.b),
                       const_cast<double*>(d.W), zero, nonfinite, m32, d.ldp32);
    } else {
      gs_csr_tile(d.rp, d.gs_val, d.gs_b, d.gs_p, row0, nrows, const_cast<double*>(d.val),
                  const_cast<double*>(d.b), nullptr, const_cast<double*>(d.W), L, zero,
                  nonfinite, m32);
    }
    if (zero) atomicOr(bad, BAD_ZERO);
    if (nonfinite) atomicOr(bad, BAD_NONFINITE);
    return;
  }
  if (!m32) return;
  if (d.kind == MAT_STENCIL) {
    const int planes = d.nz > 1 ? 7 : 5;
    if (t < nrows)
      for (int q = 0; q < planes; ++q)
        m32[(size_t)q * d.ldp32 + row0 + t] = (float)d.coef[(size_t)q * d.n + row0 + t];
  } else {
    const int k0 = d.rp[row0], k1 = d.rp[row0 + nrows];
    for (int k = k0 + t; k < k1; k += BS) m32[k] = (float)d.val[k];
  }
}

// Arguments of the GMRES engine's launches.
// Partial columns of a GMRES(m) engine: A's j+2 <= m+1 (three for the residual), then C's.
inline int gmres_partial_cols(int m) { return (m + 1 > 3 ? m + 1 : 3) + 1; }

struct GArgs {
  const SysDesc* sys;
  const int* act;        // [2][max_units]: units of the admitted systems, then their slots
  const int* n_act;      // number of entries in act
  Ctl* ctl;              // [max_systems]
  Summary* sums;         // [max_systems]: copies of the control blocks' summaries
  double* partials;      // [columns][pstride]
  int pstride;           // partials per column (the engine's tile count)
  int ccol;              // the column of C's partials, apart from A's (see batch_gmres.hip)
  int max_units;
  void* V;               // basis: m+1 columns of ldv values (double or float)
  void* w;               // ldv values
  size_t ldv;
  double zero;           // 0.0, passed at run time (see gmres.hip)
  int mixed;             // FP32 data with FP64 restarts
};

// Arguments of the mixed-precision Bi-CGSTAB engine's launches (FP32 vectors in the engine's
// row space, the FP32 matrix copy in the caller's memory).
struct MArgs {
  const SysDesc* sys;
  const int* act;        // [2][max_units]
  const int* n_act;
  BCtl* ctl;
  double* partials;      // [4][pstride], per tile
  int pstride;
  int max_units;
  float* r;              // stored residual r~
  float* rh;
  float* p[2];
  float* v[2];
  float* t;
  double* r64;           // FP64 vectors of the systems that continue in FP64
  double* rh64;
  double* p64[2];
  double* v64[2];
  double* t64;
  double* xprev;         // x at the start of the current float run (FP64)
  double delta;          // a run ends at a reduction by delta of the residual it started from
  int run_cap;           // ... or after run_cap iterations (0: no cap)
  int par;
};

// Enqueues one mixed-precision Bi-CGSTAB chunk (preparation, residual, k iterations).
hipError_t launch_bicg_mixed_chunk(MArgs a, int k, int64_t first_iter, int grid, int max_sys,
                                   hipStream_t s);

// Enqueues one GMRES chunk (one cycle of m steps for every running system, with the
// preparation, start, x update and restart launches around it) with streaming grid `grid`.
// column: the basis fits one buffer descriptor (under 2^31 bytes). nt: the admitted systems'
// cycle working set exceeds the last-level cache (non-temporal basis and plane loads, and the
// LDS-window product for FP64 stencils; the same bits).
hipError_t launch_gmres_chunk(const GArgs& a, int m, int grid, int max_sys, bool column,
                              bool nt, hipStream_t s);

// Initial control block of an admitted GMRES system.
hipError_t launch_gmres_init(Ctl* c, int maxit, int m, double tol, double eps_b, int has_w,
                             int prepare, hipStream_t s);

}  // namespace gsk
