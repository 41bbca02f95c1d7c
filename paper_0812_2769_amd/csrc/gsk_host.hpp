// Host-side interfaces between the C ABI layer (api.hip) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stddef.h>
#include <stdint.h>

#include "gsk_dev.hpp"

namespace gsk {

struct Csr {
  int n;
  int64_t nnz;
  const int* rp;
  const int* ci;
  const double* val;
};

enum : int { MAT_CSR = 0, MAT_STENCIL = 1 };

// A matrix as the solvers see it: CSR, or a structured 5/7-point stencil (coefficient planes).
struct Mat {
  int kind;
  int n;
  Csr csr;                 // MAT_CSR
  int nx, ny, nz;          // MAT_STENCIL (nz == 1: 5-point 2D)
  const double* coef;      // MAT_STENCIL: planes of n values
  int planes() const { return nz > 1 ? 7 : 5; }
  // Algorithmic bytes of one read of the matrix.
  double bytes() const {
    if (kind == MAT_STENCIL) return 8.0 * planes() * (double)n;
    return 12.0 * (double)csr.nnz + 4.0 * ((double)csr.n + 1);
  }
  CsrOp csr_op() const { return CsrOp{csr.rp, csr.ci, csr.val}; }
  StencilOp stencil_op() const { return StencilOp{coef, n, nx, ny, nz, (size_t)n}; }
};

struct SolveParams {
  int maxit;
  double tol;
  double eps_b;
  const double* weights;  // device [n] or nullptr
  int check_every;        // Bi-CGSTAB chunk length
};

struct SolveResult {
  int code;               // 0 ok, <0 error (GSK_ERR_*)
  Summary sum;
};

// Workspace carve-up: [Ctl | flags | partials | vectors...], every piece 256-byte aligned.
// The partials hold NC_MAX values per workgroup of the launch geometry.
constexpr size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
constexpr size_t kCtlBytes = align256(sizeof(Ctl));
constexpr size_t kFlagBytes = 256;
inline size_t partial_bytes(int n) {
  return align256(sizeof(double) * NC_MAX * (size_t)make_geom(n).nb);
}
inline size_t head_bytes(int n) { return kCtlBytes + kFlagBytes + partial_bytes(n); }

inline size_t vec_ld(int n) { return (size_t)((n + 63) / 64 * 64); }  // doubles, 512 B steps

struct Workspace {
  Ctl* ctl;
  int* flags;        // [0] invalid CSR, [1] zero row, [2] non-finite
  double* partials;
  double* vecs;      // method-specific vectors, each vec_ld(n) doubles
};

inline Workspace carve(void* ws, int n) {
  char* p = static_cast<char*>(ws);
  Workspace w;
  w.ctl = reinterpret_cast<Ctl*>(p);
  w.flags = reinterpret_cast<int*>(p + kCtlBytes);
  w.partials = reinterpret_cast<double*>(p + kCtlBytes + kFlagBytes);
  w.vecs = reinterpret_cast<double*>(p + head_bytes(n));
  return w;
}

size_t workspace_bytes(int method, int n, int m);
// Exact size for a given matrix (the mixed-precision GMRES keeps an FP32 copy of its values).
size_t workspace_bytes_for(const Mat& A, int method, int m);
size_t mixed_matrix_floats(const Mat& A);

// Flat validity scan of a CSR matrix (no indirect loads): row_ptr[0] == 0, non-decreasing,
// row_ptr[n] == nnz, every column index in [0, n). Sets flags[0] on failure.
hipError_t launch_clear_flags(int* flags, hipStream_t s);
hipError_t launch_validate(const Csr& A, int* flags, hipStream_t s);

hipError_t launch_gs_scale(const Csr& A, const double* b, int p, double* val_out, double* b_out,
                           double* norm, double* weight, int* flags, hipStream_t s);
hipError_t launch_spmv(const Mat& A, const double* x, double* y, hipStream_t s);
// Pack a CSR matrix with the 5/7-point pattern of an nx x ny x nz grid into coefficient
// planes; sets flags[3] if some entry is not a stencil position of its row (or repeats one).
hipError_t launch_stencil_from_csr(const Csr& A, int nx, int ny, int nz, double* coef,
                                   int* flags, hipStream_t s);

SolveResult gmres_solve(const Mat& A, const double* b, double* x, int m,
                        const SolveParams& prm, void* ws, hipStream_t s);
SolveResult arnoldi_run(const Mat& A, const double* r0, int m, double* V, int64_t ldv,
                        double* H, void* ws, double eps_b, hipStream_t s);
SolveResult bicgstab_solve(const Mat& A, const double* b, double* x, const SolveParams& prm,
                           void* ws, hipStream_t s);
// Bi-CGSTAB without allocation: the workspace is a file-scope device array of kNoAllocBytes
// (its address on the current device from noalloc_scratch).
constexpr size_t kNoAllocBytes = size_t(32) << 20;
void* noalloc_scratch(hipError_t* err);
SolveResult bicgstab_solve_noalloc(const Mat& A, const double* b, double* x,
                                   const SolveParams& prm, void* scratch_ptr, hipStream_t s);
// GMRES(m) with FP32 Arnoldi cycles and FP64 restarts (iterative refinement).
SolveResult gmres_mixed_solve(const Mat& A, const double* b, double* x, int m,
                              const SolveParams& prm, void* ws, hipStream_t s);

// The batch engine (batch.hip, batch_gmres.hip): many independent systems share every launch.
struct Engine;
struct EngineDone {
  int64_t tag;
  Summary sum;
};
// Last-level cache of the device (256 MB of Infinity Cache on MI355X): working sets above it
// are streamed from HBM once per launch, and loads or stores that are not reused within the
// launch then take the non-temporal policy.
constexpr double kStreamBytes = 256.0 * (1 << 20);

// measure.hip: the measurement hook's stream-mix kernel (0, -1 unsupported mix, -5 HIP failure)
int stream_mix_ms(int reads, int writes, int64_t n, double* buf, int reps, float* best_ms,
                  hipStream_t s);

struct EngineConfig {
  int64_t max_rows;
  int max_sys;
  int method;        // 0 Bi-CGSTAB, 1 GMRES(m)
  int m;             // GMRES restart length
  bool mixed;        // FP32 storage with FP64 refinement (GMRES cycles or Bi-CGSTAB runs)
  int check_every;   // Bi-CGSTAB: iterations per chunk
  bool use_graph;
  double delta;      // mixed Bi-CGSTAB: reduction that ends a run (refinement step)
  int run_cap = 0;   // mixed Bi-CGSTAB: iterations that end a run (0: no cap)
  int units;         // FP64 Bi-CGSTAB: 256-row tiles per workgroup (1 or 2; 0 = 1)
  // FP64 Bi-CGSTAB: launch shape per size class (kClass2D, kClass3DSmall, kClass3DLarge), each
  // one of the kShape* codes; all 0: one class, shaped by `units`
  int class_shape[3] = {0, 0, 0};
};
// Size classes of an FP64 Bi-CGSTAB engine with per-class launch shapes: 2D stencils and CSR
// matrices; 3D stencils of fewer than kClassLargeRows rows; larger 3D stencils.
enum : int { kClass2D = 0, kClass3DSmall = 1, kClass3DLarge = 2, kClassCount = 3 };
constexpr int kClassLargeRows = 1 << 18;
// Launch shapes of a class (rows are handed out in pairs of tiles): P and S one tile per
// workgroup, U one tile; P and S two tiles per workgroup (both tiles' loads in flight), U one
// tile; P and S two tiles, U a unit's two tiles in turn.
enum : int { kShapeTile = 1, kShapePairTileU = 2, kShapePair = 3 };
size_t engine_workspace_bytes(const EngineConfig& cfg);
// 0 ok, -4 workspace too small, -1 invalid arguments, -5 HIP failure.
int engine_create(void* ws, size_t ws_bytes, const EngineConfig& cfg, hipStream_t s,
                  Engine** out);
void engine_destroy(Engine* e);
// Optional stage of a submitted system run by its first chunk. p > 0: GS(p), with outputs of
// the scaled matrix values (CSR values or planes, same layout as the input), b and (p != 2)
// stop weights. mat32 (mixed GMRES engines, required there): the FP32 copy of the scaled
// matrix (planes of stride ldp32, or nnz values).
struct GsStage {
  int p;
  double* val_out;
  double* b_out;
  double* weight_out;
  float* mat32;
  size_t ldp32;
};
// 0 admitted, 1 no free slot or rows (try again after a poll), -1 invalid arguments (a mixed
// engine without an FP32 matrix buffer), -5 HIP failure.
int engine_submit(Engine* e, const Mat& A, const double* b, double* x, const SolveParams& prm,
                  int64_t tag, const GsStage* gs = nullptr);
int engine_run(Engine* e, int chunks);
int engine_poll(Engine* e, bool wait, EngineDone* out, int max_out, int* n_out);
void engine_usage(const Engine* e, int* active, int64_t* free_rows, int64_t* largest_free_rows);

// Small pinned host buffer for status read-back (one per thread, allocated on first use).
Summary* pinned_summaries();

// How far ahead of the device the host enqueues. The solvers enqueue a cycle (GMRES) or a
// chunk of iterations (Bi-CGSTAB) without waiting, one ahead of the status the host has read;
// launches enqueued past the end of a solve find it finished and store nothing, but they
// still take time. Once the residual history predicts that the work in flight may finish the
// solve (the last relative residual times the last reduction factor is within `margin` of
// the tolerance), or the iteration cap is near, the pacer turns cautious and stays so: the
// host then waits for each result before it enqueues more, and enqueues in smaller pieces.
struct Pacer {
  double tol;
  long maxit;
  int span;               // iterations one cycle or chunk can add
  double margin = 4.0;
  double last = -1.0;
  bool cautious = false;
  void update(int iters, double relres) {
    if (last > 0.0 && relres > 0.0) {
      const double ratio = relres < last ? relres / last : 1.0;
      if (relres * ratio < margin * tol) cautious = true;
    }
    if (relres < margin * tol || (long)iters + 2L * span >= maxit) cautious = true;
    last = relres;
  }
};

// Measurement hook (gsk_probe_begin / gsk_probe_end). While a kernel class is selected, every
// sample_every-th launch of that class gets a slot number and a pair of HIP events that the
// launch itself carries (hipExtLaunchKernel: the events take the dispatch's own start and end
// times, with no marker packets around it), and the kernel records its algorithmic bytes in
// the slot if it did work. At the end of each solve the working launches' durations and bytes
// are added to the totals.
void probe_solve_begin();                  // a new solve starts: slots restart at 0
int probe_slot(int kernel_class);          // -1 if this launch is not timed
// The batch engine samples whole chunks: probe_every(c) is the sampling period while class c
// is selected (0 otherwise), and probe_slot_all(c) hands a slot to every launch of a sampled
// chunk.
int probe_every(int kernel_class);
int probe_slot_all(int kernel_class);
bool probe_pair(int slot, hipEvent_t* start, hipEvent_t* stop);   // events for a timed launch
void probe_collect(const ProbeSlots* device_slots, hipStream_t s);

// Launches kernel(args...) on s with BS-wide workgroups; a launch with a probe slot carries
// that slot's timing events.
template <class F, class... Args>
inline void launch_probed(F kernel, dim3 grid, hipStream_t s, int slot, Args... args) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (slot >= 0 && !probe_pair(slot, &e0, &e1)) e0 = e1 = nullptr;
  hipExtLaunchKernelGGL(kernel, grid, dim3(BS), 0, s, e0, e1, 0, args...);
}

}  // namespace gsk
