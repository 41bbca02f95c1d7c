// C ABI of the gsk library: argument checks, workspace sizing, error reporting.
// The declarations and their documentation live in include/gsk.h.
#include <float.h>
#include <stdarg.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "gsk.h"
#include "gsk_host.hpp"

namespace gsk {

namespace {
thread_local std::string g_err;

// A named range on the calling thread for rocprofv3's marker trace (--marker-trace): one per
// solve, GS(p) call and engine chunk run or poll. Without a profiler attached the calls cost a
// function call each.
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

struct Pinned {
  Summary sum[2];
  int flags[4];
};

// A thread's pinned status block: allocated on the thread's first solve, freed when the thread
// exits (serving lanes and other worker threads come and go).
struct PinnedHolder {
  Pinned* p = nullptr;
  ~PinnedHolder() {
    if (p) (void)hipHostFree(p);
  }
};
thread_local PinnedHolder g_pinned;

int set_err(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int set_err(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_err(hipError_t e, const char* what) {
  return set_err(GSK_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

Pinned* pinned() {
  if (!g_pinned.p) {
    void* p = nullptr;
    if (hipHostMalloc(&p, sizeof(Pinned), hipHostMallocDefault) != hipSuccess) return nullptr;
    g_pinned.p = static_cast<Pinned*>(p);
  }
  return g_pinned.p;
}

int check_csr(const gsk_csr* A) {
  if (!A) return set_err(GSK_ERR_INVALID_ARG, "matrix is NULL");
  if (A->n < 1) return set_err(GSK_ERR_INVALID_ARG, "n = %d must be >= 1", (int)A->n);
  if (A->nnz < 0 || A->nnz > (int64_t)INT32_MAX)
    return set_err(GSK_ERR_INVALID_ARG, "nnz = %lld out of range", (long long)A->nnz);
  if (!A->row_ptr) return set_err(GSK_ERR_INVALID_ARG, "row_ptr is NULL");
  if (A->nnz > 0 && (!A->col_idx || !A->val))
    return set_err(GSK_ERR_INVALID_ARG, "col_idx/val is NULL");
  return GSK_OK;
}

int check_ws(void* ws, size_t ws_bytes, size_t need) {
  if (!ws) return set_err(GSK_ERR_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
    return set_err(GSK_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  if (ws_bytes < need)
    return set_err(GSK_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, need);
  return GSK_OK;
}

Csr to_csr(const gsk_csr* A) {
  return Csr{A->n, A->nnz, A->row_ptr, A->col_idx, A->val};
}

int check_matrix(const gsk_matrix* A, Mat& out) {
  if (!A) return set_err(GSK_ERR_INVALID_ARG, "matrix is NULL");
  out = Mat{};
  if (A->kind == GSK_MATRIX_CSR) {
    int rc = check_csr(&A->csr);
    if (rc) return rc;
    out.kind = MAT_CSR;
    out.n = A->csr.n;
    out.csr = to_csr(&A->csr);
    return GSK_OK;
  }
  if (A->kind == GSK_MATRIX_STENCIL) {
    const gsk_stencil& S = A->stencil;
    if (S.nx < 2 || S.ny < 2 || S.nz < 1)
      return set_err(GSK_ERR_INVALID_ARG, "stencil grid %d x %d x %d: need nx, ny >= 2, nz >= 1",
                     (int)S.nx, (int)S.ny, (int)S.nz);
    const int64_t n = (int64_t)S.nx * S.ny * S.nz;
    if (n > INT32_MAX) return set_err(GSK_ERR_INVALID_ARG, "stencil grid too large");
    if (!S.coef) return set_err(GSK_ERR_INVALID_ARG, "stencil coef is NULL");
    out.kind = MAT_STENCIL;
    out.n = (int)n;
    out.nx = S.nx;
    out.ny = S.ny;
    out.nz = S.nz;
    out.coef = S.coef;
    return GSK_OK;
  }
  return set_err(GSK_ERR_INVALID_ARG, "unknown matrix kind %d", (int)A->kind);
}

int params_from(const gsk_options* opt, SolveParams& prm, double tol) {
  gsk_options o;
  gsk_default_options(&o);
  if (opt) o = *opt;
  if (!(tol > 0.0) || !isfinite(tol)) return set_err(GSK_ERR_INVALID_ARG, "tol must be > 0");
  if (o.maxit < 0) return set_err(GSK_ERR_INVALID_ARG, "maxit must be >= 0");
  if (!(o.breakdown_eps >= 0.0) || !isfinite(o.breakdown_eps))
    return set_err(GSK_ERR_INVALID_ARG, "breakdown_eps must be finite and >= 0");
  if (o.check_every < 1 || o.check_every > 256)
    return set_err(GSK_ERR_INVALID_ARG, "check_every must be in [1, 256]");
  prm.maxit = o.maxit;
  prm.tol = tol;
  prm.eps_b = o.breakdown_eps;
  prm.weights = o.stop_weights;
  prm.check_every = o.check_every;
  return GSK_OK;
}

void fill_info(gsk_info* info, const Summary& s) {
  if (!info) return;
  info->iters = s.iters;
  info->restarts = s.restarts;
  info->status = s.status;
  info->half_step = s.half;
  info->verify_failures = s.fails;
  info->breakdown_test = s.status == GSK_BREAKDOWN ? s.brk : 0;
  info->fp64_from = s.fp64_from;
  info->reserved = 0;
  info->relres_recursive = s.relres_rec;
  info->relres_true = s.relres_true;
}

struct Probe {
  std::mutex mu;
  std::atomic<int> cls{0};
  int every = 1;
  long long seen = 0;      // launches of the class since gsk_probe_begin
  int next_slot = 0;       // slots handed out in the current solve
  struct Timed {
    hipEvent_t start, stop;
    int slot;
  };
  std::vector<hipEvent_t> pool;
  std::vector<Timed> timed;
  double total_ms = 0.0;
  long long launches = 0;
  long long busy = 0;
  double bytes = 0.0;
};

Probe& probe_state() {
  static Probe p;
  return p;
}

hipEvent_t take_event(Probe& p) {
  if (!p.pool.empty()) {
    hipEvent_t e = p.pool.back();
    p.pool.pop_back();
    return e;
  }
  // Timing events without the system-scope fence a default event performs when it is
  // recorded; only their timestamps are used.
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

void recycle(Probe& p) {
  for (auto& t : p.timed) {
    p.pool.push_back(t.start);
    p.pool.push_back(t.stop);
  }
  p.timed.clear();
}

}  // namespace

void probe_solve_begin() {
  Probe& p = probe_state();
  if (p.cls.load(std::memory_order_relaxed) == KC_NONE) return;
  std::lock_guard<std::mutex> g(p.mu);
  recycle(p);   // pairs of an earlier solve that was never collected (an error path)
  p.next_slot = 0;
}

int probe_slot(int kernel_class) {
  Probe& p = probe_state();
  if (p.cls.load(std::memory_order_relaxed) != kernel_class) return -1;
  std::lock_guard<std::mutex> g(p.mu);
  const long long k = p.seen++;
  if (k % p.every != 0 || p.next_slot >= PROBE_SLOTS) return -1;
  return p.next_slot++;
}

int probe_every(int kernel_class) {
  Probe& p = probe_state();
  if (p.cls.load(std::memory_order_relaxed) != kernel_class) return 0;
  std::lock_guard<std::mutex> g(p.mu);
  return p.every;
}

int probe_slot_all(int kernel_class) {
  Probe& p = probe_state();
  if (p.cls.load(std::memory_order_relaxed) != kernel_class) return -1;
  std::lock_guard<std::mutex> g(p.mu);
  if (p.next_slot >= PROBE_SLOTS) return -1;
  return p.next_slot++;
}

bool probe_pair(int slot, hipEvent_t* start, hipEvent_t* stop) {
  Probe& p = probe_state();
  std::lock_guard<std::mutex> g(p.mu);
  hipEvent_t a = take_event(p);
  hipEvent_t b = a ? take_event(p) : nullptr;
  if (!b) {
    if (a) p.pool.push_back(a);
    return false;
  }
  p.timed.push_back(Probe::Timed{a, b, slot});
  *start = a;
  *stop = b;
  return true;
}

// After a solve has synchronised its stream: add the durations and bytes of the timed
// launches that did work (their slot holds their algorithmic bytes; zero means the launch
// returned at once).
void probe_collect(const ProbeSlots* device_slots, hipStream_t s) {
  Probe& p = probe_state();
  if (p.cls.load(std::memory_order_relaxed) == KC_NONE) return;
  std::lock_guard<std::mutex> g(p.mu);
  if (p.timed.empty()) return;
  std::vector<double> bytes((size_t)p.next_slot, 0.0);
  if (p.next_slot > 0 &&
      (hipMemcpyAsync(bytes.data(), device_slots->bytes, sizeof(double) * (size_t)p.next_slot,
                      hipMemcpyDeviceToHost, s) != hipSuccess ||
       hipStreamSynchronize(s) != hipSuccess)) {
    recycle(p);
    return;
  }
  for (auto& t : p.timed) {
    p.launches += 1;
    const double b = (t.slot >= 0 && t.slot < p.next_slot) ? bytes[(size_t)t.slot] : 0.0;
    if (b <= 0.0) continue;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, t.start, t.stop) != hipSuccess) continue;
    p.busy += 1;
    p.total_ms += ms;
    p.bytes += b;
  }
  recycle(p);
}

Summary* pinned_summaries() {
  Pinned* p = pinned();
  return p ? p->sum : nullptr;
}

size_t workspace_bytes(int method, int n, int m) {
  if (n < 1) return 0;
  const size_t ld = vec_ld(n) * sizeof(double);
  const size_t head = head_bytes(n);
  switch (method) {
    case GSK_METHOD_GS:
      return kCtlBytes + kFlagBytes;
    case GSK_METHOD_GMRES:
      if (m < 1 || m > GSK_MAX_RESTART) return 0;
      return head + (size_t)(m + 2) * ld;
    case GSK_METHOD_ARNOLDI:
      if (m < 1 || m > GSK_MAX_RESTART) return 0;
      return head + ld;
    case GSK_METHOD_BICGSTAB:
      return head + 7 * ld;
    case GSK_METHOD_GMRES_MIXED:   // sized for a 7-point stencil matrix
      if (m < 1 || m > GSK_MAX_RESTART) return 0;
      return head + align256(sizeof(float) * 7 * vec_ld(n)) +
             (size_t)(m + 2) * vec_ld(n) * sizeof(float);
    default:
      return 0;
  }
}

size_t workspace_bytes_for(const Mat& A, int method, int m) {
  if (method != GSK_METHOD_GMRES_MIXED) return workspace_bytes(method, A.n, m);
  if (A.n < 1 || m < 1 || m > GSK_MAX_RESTART) return 0;
  return head_bytes(A.n) + align256(sizeof(float) * mixed_matrix_floats(A)) +
         (size_t)(m + 2) * vec_ld(A.n) * sizeof(float);
}

}  // namespace gsk

using namespace gsk;

static_assert(GSK_MAX_RESTART == gsk::MMAX, "restart limit mismatch");

extern "C" {

void gsk_default_options(gsk_options* opt) {
  if (!opt) return;
  opt->maxit = 10000;
  opt->breakdown_eps = 1e-16 * DBL_EPSILON;
  opt->stop_weights = nullptr;
  opt->check_every = 8;
}

size_t gsk_workspace_bytes(int32_t method, int32_t n, int32_t m) {
  return gsk::workspace_bytes(method, n, m);
}

size_t gsk_workspace_bytes_for(const gsk_matrix* A, int32_t method, int32_t m) {
  g_err.clear();
  Mat M;
  if (check_matrix(A, M)) return 0;   // the reason is left in gsk_last_error()
  return gsk::workspace_bytes_for(M, method, m);
}

int gsk_version(void) { return GSK_VERSION; }

int gsk_probe_begin(int32_t kernel_class, int32_t sample_every) {
  g_err.clear();
  if (kernel_class < GSK_KCLASS_GMRES_A || kernel_class > GSK_KCLASS_BATCH_U)
    return set_err(GSK_ERR_INVALID_ARG, "unknown kernel class %d", (int)kernel_class);
  if (sample_every < 1) return set_err(GSK_ERR_INVALID_ARG, "sample_every must be >= 1");
  Probe& p = probe_state();
  std::lock_guard<std::mutex> g(p.mu);
  p.total_ms = 0.0;
  p.launches = 0;
  p.busy = 0;
  p.bytes = 0.0;
  p.seen = 0;
  p.next_slot = 0;
  p.every = sample_every;
  recycle(p);
  p.cls.store(kernel_class, std::memory_order_relaxed);
  return GSK_OK;
}

static bool stream_mix_supported(int32_t reads, int32_t writes) {
  return (reads == 1 && (writes == 0 || writes == 1)) || (reads == 6 && writes == 2) ||
         (reads == 9 && writes == 1) || (reads == 11 && writes == 2);
}

size_t gsk_stream_mix_bytes(int32_t reads, int32_t writes, int64_t n) {
  if (!stream_mix_supported(reads, writes) || n < 1 || n > ((int64_t)1 << 34)) return 0;
  const int64_t tiles = (n + gsk::BS - 1) / gsk::BS;
  return sizeof(double) * ((size_t)(reads + writes) * (size_t)n + (size_t)((tiles + 7) / 8 * 8));
}

int gsk_stream_mix_ms(int32_t reads, int32_t writes, int64_t n, void* buf, size_t buf_bytes,
                      int32_t reps, float* best_ms, void* stream) {
  g_err.clear();
  const size_t need = gsk_stream_mix_bytes(reads, writes, n);
  if (need == 0) return set_err(GSK_ERR_INVALID_ARG, "unsupported mix or n");
  if (!buf || !best_ms || reps < 1 || reps > 1000)
    return set_err(GSK_ERR_INVALID_ARG, "buf, best_ms or reps (1..1000)");
  if (buf_bytes < need) return set_err(GSK_ERR_WORKSPACE, "buf needs %zu bytes", need);
  if ((int64_t)((n + gsk::BS - 1) / gsk::BS) > (int64_t)INT32_MAX / 2)
    return set_err(GSK_ERR_INVALID_ARG, "n too large");
  const int rc = gsk::stream_mix_ms(reads, writes, n, static_cast<double*>(buf), reps, best_ms,
                                    static_cast<hipStream_t>(stream));
  if (rc) return set_err(GSK_ERR_DEVICE, "stream mix: HIP failure");
  return GSK_OK;
}

int gsk_probe_end(gsk_probe_result* out) {
  g_err.clear();
  Probe& p = probe_state();
  hipError_t e = hipDeviceSynchronize();
  std::lock_guard<std::mutex> g(p.mu);
  recycle(p);
  if (out) {
    out->launches = p.launches;
    out->busy_launches = p.busy;
    out->total_ms = p.total_ms;
    out->bytes = p.bytes;
  }
  p.cls.store(0, std::memory_order_relaxed);
  if (e != hipSuccess) return hip_err(e, "probe end");
  return GSK_OK;
}

const char* gsk_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------------------
// Engine (batched Bi-CGSTAB)
// ---------------------------------------------------------------------------------------
struct gsk_engine {
  gsk::Engine* impl;
  int64_t max_rows;
  int32_t max_systems;
  int32_t method;
  int32_t precision;
};

static int engine_cfg(const gsk_engine_config* c, gsk::EngineConfig& cfg) {
  if (!c) return set_err(GSK_ERR_INVALID_ARG, "config is NULL");
  if (c->max_rows < 1 || c->max_rows > ((int64_t)1 << 40) || c->max_systems < 1 ||
      c->max_systems > (1 << 20))
    return set_err(GSK_ERR_INVALID_ARG, "max_rows and max_systems must be positive");
  if (c->method != GSK_METHOD_BICGSTAB && c->method != GSK_METHOD_GMRES)
    return set_err(GSK_ERR_INVALID_ARG, "method must be GSK_METHOD_BICGSTAB or GSK_METHOD_GMRES");
  if (c->precision != GSK_PRECISION_FP64 && c->precision != GSK_PRECISION_MIXED)
    return set_err(GSK_ERR_INVALID_ARG, "unknown precision");
  const bool gmres = c->method == GSK_METHOD_GMRES;
  const double delta = c->inner_reduction == 0.0 ? 1e-6 : c->inner_reduction;
  if (!gmres && c->precision == GSK_PRECISION_MIXED && !(delta > 0.0 && delta < 1.0))
    return set_err(GSK_ERR_INVALID_ARG, "inner_reduction must be in (0, 1)");
  if (gmres && (c->m < 1 || c->m > GSK_MAX_RESTART))
    return set_err(GSK_ERR_INVALID_ARG, "m must be in [1, %d]", GSK_MAX_RESTART);
  if (!gmres && (c->check_every < 1 || c->check_every > 256))
    return set_err(GSK_ERR_INVALID_ARG, "check_every must be in [1, 256]");
  cfg.max_rows = c->max_rows;
  cfg.max_sys = c->max_systems;
  cfg.method = gmres ? 1 : 0;
  cfg.m = gmres ? c->m : 0;
  cfg.mixed = c->precision == GSK_PRECISION_MIXED;
  cfg.check_every = gmres ? 0 : c->check_every;
  cfg.use_graph = (c->flags & GSK_ENGINE_GRAPH) != 0;
  cfg.delta = delta;
  if (c->run_cap < -1) return set_err(GSK_ERR_INVALID_ARG, "run_cap must be >= -1");
  cfg.run_cap = c->run_cap == 0 ? 1000 : c->run_cap < 0 ? 0 : c->run_cap;
  if (c->tile_units < 0 || c->tile_units > 2 ||
      (c->tile_units == 2 && (gmres || c->precision != GSK_PRECISION_FP64)))
    return set_err(GSK_ERR_INVALID_ARG, "tile_units must be 0 or 1 (or 2 for FP64 Bi-CGSTAB)");
  cfg.units = c->tile_units;
  if (c->class_shapes != 0) {
    if (gmres || c->precision != GSK_PRECISION_FP64)
      return set_err(GSK_ERR_INVALID_ARG, "class_shapes applies to FP64 Bi-CGSTAB engines only");
    if ((uint32_t)c->class_shapes >> 12)
      return set_err(GSK_ERR_INVALID_ARG, "class_shapes has bits beyond its three classes");
    for (int k = 0; k < 3; ++k) {
      const int code = (c->class_shapes >> (4 * k)) & 15;
      if (code > 3) return set_err(GSK_ERR_INVALID_ARG, "class_shapes: shape codes are 0..3");
      cfg.class_shape[k] = code;
    }
  }
  return GSK_OK;
}

size_t gsk_engine_workspace_bytes_ex(const gsk_engine_config* c) {
  gsk::EngineConfig cfg;
  const std::string saved = g_err;
  const int rc = engine_cfg(c, cfg);
  g_err = saved;
  return rc ? 0 : gsk::engine_workspace_bytes(cfg);
}

size_t gsk_engine_workspace_bytes(int64_t max_rows, int32_t max_systems) {
  const gsk_engine_config c{max_rows, max_systems, GSK_METHOD_BICGSTAB, 0, GSK_PRECISION_FP64,
                            8, 0, 0, 0.0};
  return gsk_engine_workspace_bytes_ex(&c);
}

int gsk_engine_create_ex(const gsk_engine_config* c, void* ws, size_t ws_bytes, void* stream,
                         gsk_engine** out) {
  g_err.clear();
  if (!out) return set_err(GSK_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  gsk::EngineConfig cfg;
  int rc = engine_cfg(c, cfg);
  if (rc) return rc;
  if (cfg.use_graph && (!stream || (cfg.method == 0 && (cfg.check_every & 1))))
    return set_err(GSK_ERR_INVALID_ARG,
                   "GSK_ENGINE_GRAPH needs a non-default stream (and, for Bi-CGSTAB, an even "
                   "check_every)");
  rc = check_ws(ws, ws_bytes, gsk::engine_workspace_bytes(cfg));
  if (rc) return rc;
  gsk::Engine* impl = nullptr;
  rc = gsk::engine_create(ws, ws_bytes, cfg, static_cast<hipStream_t>(stream), &impl);
  if (rc == -4) return set_err(GSK_ERR_WORKSPACE, "engine workspace too small");
  if (rc == -1) return set_err(GSK_ERR_INVALID_ARG, "invalid engine configuration");
  if (rc) return set_err(GSK_ERR_DEVICE, "engine: pinned host buffers or events unavailable");
  *out = new gsk_engine{impl, c->max_rows, c->max_systems, c->method, c->precision};
  return GSK_OK;
}

int gsk_engine_create(void* ws, size_t ws_bytes, int64_t max_rows, int32_t max_systems,
                      int32_t check_every, int32_t flags, void* stream, gsk_engine** out) {
  const gsk_engine_config c{max_rows, max_systems, GSK_METHOD_BICGSTAB, 0, GSK_PRECISION_FP64,
                            check_every, flags, 0, 0.0};
  return gsk_engine_create_ex(&c, ws, ws_bytes, stream, out);
}

int gsk_engine_submit_ex(gsk_engine* e, const gsk_engine_request* r) {
  g_err.clear();
  if (!e) return set_err(GSK_ERR_INVALID_ARG, "engine is NULL");
  if (!r) return set_err(GSK_ERR_INVALID_ARG, "request is NULL");
  Mat M;
  int rc = check_matrix(r->A, M);
  if (rc) return rc;
  if (!r->b || !r->x) return set_err(GSK_ERR_INVALID_ARG, "b or x is NULL");
  const int p = r->gs_p;
  if (p < 0) return set_err(GSK_ERR_INVALID_ARG, "gs_p must be >= 0");
  if (p > 0) {
    if (!r->val_out || !r->b_out) return set_err(GSK_ERR_INVALID_ARG, "GS outputs are NULL");
    if (p != 2 && !r->stop_weight_out)
      return set_err(GSK_ERR_INVALID_ARG, "p != 2 needs stop_weight_out");
    if (r->opt && r->opt->stop_weights)
      return set_err(GSK_ERR_INVALID_ARG, "opt->stop_weights must be NULL with a GS stage");
  }
  const bool mixed = e->precision == GSK_PRECISION_MIXED;
  if (mixed) {
    if (!r->mat32) return set_err(GSK_ERR_INVALID_ARG, "a mixed engine needs mat32");
    if (M.kind == gsk::MAT_STENCIL && r->mat32_ld < M.n)
      return set_err(GSK_ERR_INVALID_ARG, "mat32_ld must be >= n");
  } else if (r->mat32) {
    return set_err(GSK_ERR_INVALID_ARG, "mat32 is only for mixed-precision engines");
  }
  SolveParams prm;
  rc = params_from(r->opt, prm, r->tol);
  if (rc) return rc;
  gsk::GsStage gs{p, r->val_out, r->b_out, p != 2 ? r->stop_weight_out : nullptr, r->mat32,
                  (size_t)(r->mat32_ld > 0 ? r->mat32_ld : 0)};
  rc = gsk::engine_submit(e->impl, M, r->b, r->x, prm, r->tag,
                          (p > 0 || mixed) ? &gs : nullptr);
  if (rc == 1) return GSK_FULL;
  if (rc == -1) return set_err(GSK_ERR_INVALID_ARG, "invalid request");
  if (rc == -6)
    return set_err(GSK_ERR_INVALID_ARG, "tag %lld is already in flight in this engine",
                   (long long)r->tag);
  if (rc) return set_err(GSK_ERR_DEVICE, "engine submit: HIP failure");
  return GSK_OK;
}

int gsk_engine_submit(gsk_engine* e, const gsk_matrix* A, const double* b, double* x,
                      double tol, const gsk_options* opt, int64_t tag) {
  const gsk_engine_request r{A, b, x, tol, opt, tag, 0, nullptr, nullptr, nullptr, nullptr, 0};
  return gsk_engine_submit_ex(e, &r);
}

int gsk_engine_submit_gs(gsk_engine* e, const gsk_matrix* A, const double* b, int32_t p,
                         double* val_out, double* b_out, double* stop_weight_out, double* x,
                         double tol, const gsk_options* opt, int64_t tag) {
  if (p < 1) {
    g_err.clear();
    return set_err(GSK_ERR_INVALID_ARG, "p must be >= 1");
  }
  const gsk_engine_request r{A, b, x, tol, opt, tag, p, val_out, b_out, stop_weight_out,
                             nullptr, 0};
  return gsk_engine_submit_ex(e, &r);
}

int gsk_engine_run(gsk_engine* e, int32_t chunks) {
  const Range range("gsk_engine_run");
  g_err.clear();
  if (!e) return set_err(GSK_ERR_INVALID_ARG, "engine is NULL");
  if (chunks < 0) return set_err(GSK_ERR_INVALID_ARG, "chunks must be >= 0");
  if (chunks == 0) return GSK_OK;
  if (gsk::engine_run(e->impl, chunks))
    return set_err(GSK_ERR_DEVICE, "engine run: HIP failure (%s)",
                   hipGetErrorString(hipGetLastError()));
  return GSK_OK;
}

int gsk_engine_poll(gsk_engine* e, int32_t wait, gsk_result* out, int32_t max_out,
                    int32_t* n_out) {
  const Range range("gsk_engine_poll");
  g_err.clear();
  if (!e || !n_out || (max_out > 0 && !out) || max_out < 0)
    return set_err(GSK_ERR_INVALID_ARG, "engine, out or n_out invalid");
  *n_out = 0;
  std::vector<gsk::EngineDone> done((size_t)(max_out > 0 ? max_out : 0));
  int n = 0;
  if (gsk::engine_poll(e->impl, wait != 0, done.data(), max_out, &n))
    return set_err(GSK_ERR_DEVICE, "engine poll: HIP failure");
  for (int i = 0; i < n; ++i) {
    out[i].tag = done[i].tag;
    fill_info(&out[i].info, done[i].sum);
  }
  *n_out = n;
  return GSK_OK;
}

int gsk_engine_get_usage(gsk_engine* e, gsk_engine_usage* u) {
  g_err.clear();
  if (!e || !u) return set_err(GSK_ERR_INVALID_ARG, "engine or usage is NULL");
  int active = 0;
  int64_t free_rows = 0, largest = 0;
  gsk::engine_usage(e->impl, &active, &free_rows, &largest);
  u->active = active;
  u->max_systems = e->max_systems;
  u->max_rows = e->max_rows;
  u->free_rows = free_rows;
  u->largest_free_rows = largest;
  return GSK_OK;
}

int gsk_engine_destroy(gsk_engine* e) {
  g_err.clear();
  if (!e) return GSK_OK;
  gsk::engine_destroy(e->impl);
  delete e;
  return GSK_OK;
}

static int64_t batch_rows(int32_t count, const int32_t* n) {
  int64_t rows = 0;
  for (int32_t i = 0; i < count; ++i) {
    if (n[i] < 1) return -1;
    rows += ((int64_t)n[i] + BS - 1) / BS * BS;
  }
  return rows;
}

size_t gsk_bicgstab_batch_workspace_bytes(int32_t count, const int32_t* n) {
  if (count < 1 || !n) return 0;
  const int64_t rows = batch_rows(count, n);
  if (rows < 1) return 0;
  return gsk_engine_workspace_bytes(rows, count);
}

int gsk_bicgstab_batch(int32_t count, const gsk_matrix* A, const double* const* b,
                       double* const* x, double tol, const gsk_options* opt, gsk_info* info,
                       void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (count < 1 || !A || !b || !x || !info)
    return set_err(GSK_ERR_INVALID_ARG, "count < 1 or a NULL array");
  std::vector<int32_t> n(count);
  for (int32_t i = 0; i < count; ++i) {
    Mat M;
    int rc = check_matrix(&A[i], M);
    if (rc) return rc;
    if (!b[i] || !x[i]) return set_err(GSK_ERR_INVALID_ARG, "b[%d] or x[%d] is NULL", i, i);
    n[i] = M.n;
  }
  SolveParams prm;
  int rc = params_from(opt, prm, tol);
  if (rc) return rc;
  const int64_t rows = batch_rows(count, n.data());
  const gsk::EngineConfig cfg{rows, count, 0, 0, false, prm.check_every, false, 1e-6, 1};
  rc = check_ws(ws, ws_bytes, gsk::engine_workspace_bytes(cfg));
  if (rc) return rc;
  gsk::Engine* e = nullptr;
  if (gsk::engine_create(ws, ws_bytes, cfg, static_cast<hipStream_t>(stream), &e))
    return set_err(GSK_ERR_DEVICE, "batch: engine creation failed");
  for (int32_t i = 0; i < count; ++i) {
    Mat M;
    check_matrix(&A[i], M);
    if (gsk::engine_submit(e, M, b[i], x[i], prm, i) != 0) {
      gsk::engine_destroy(e);
      return set_err(GSK_ERR_DEVICE, "batch: submission failed");
    }
  }
  std::vector<gsk::EngineDone> done(count);
  std::vector<char> seen(count, 0);
  int left = count, bad = 0;
  // Every system finishes within 4 maxit + 16 chunks (as in gsk_bicgstab).
  const long max_chunks = (long)prm.maxit * 4 + 16;
  for (long ch = 0; ch <= max_chunks && left > 0; ++ch) {
    int got = 0;
    if (gsk::engine_run(e, 1) || gsk::engine_poll(e, true, done.data(), count, &got)) {
      gsk::engine_destroy(e);
      return set_err(GSK_ERR_DEVICE, "batch: HIP failure");
    }
    for (int i = 0; i < got; ++i) {
      const int k = (int)done[i].tag;
      fill_info(&info[k], done[i].sum);
      seen[k] = 1;
      if (done[i].sum.status < 0) bad = 1;
    }
    left -= got;
  }
  gsk::engine_destroy(e);
  if (left > 0) return set_err(GSK_ERR_DEVICE, "batch: systems did not finish");
  if (bad)
    return set_err(GSK_ERR_INVALID_ARG,
                   "a system's CSR structure is invalid (its info.status is negative)");
  return GSK_OK;
}

int gsk_gs_scale(const gsk_csr* A, const double* b, int32_t p, double* val_out, double* b_out,
                 double* row_norm, double* stop_weight, void* ws, size_t ws_bytes,
                 void* stream) {
  const Range range("gsk_gs_scale");
  g_err.clear();
  int rc = check_csr(A);
  if (rc) return rc;
  if (p < 1) return set_err(GSK_ERR_INVALID_ARG, "p = %d must be >= 1", (int)p);
  if (!b || !b_out || (A->nnz > 0 && !val_out))
    return set_err(GSK_ERR_INVALID_ARG, "b, b_out or val_out is NULL");
  rc = check_ws(ws, ws_bytes, gsk::workspace_bytes(GSK_METHOD_GS, A->n, 0));
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace W = carve(ws, A->n);
  Csr C = to_csr(A);
  hipError_t e;
  if ((e = launch_clear_flags(W.flags, s)) != hipSuccess) return hip_err(e, "clear flags");
  if ((e = launch_validate(C, W.flags, s)) != hipSuccess) return hip_err(e, "validate");
  if ((e = launch_gs_scale(C, b, p, val_out, b_out, row_norm, stop_weight, W.flags, s)) !=
      hipSuccess)
    return hip_err(e, "gs_scale launch");
  Pinned* pin = pinned();
  if (!pin) return set_err(GSK_ERR_DEVICE, "pinned host buffer allocation failed");
  if ((e = hipMemcpyAsync(pin->flags, W.flags, 4 * sizeof(int), hipMemcpyDeviceToHost, s)) !=
      hipSuccess)
    return hip_err(e, "flag read-back");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_err(e, "gs_scale");
  if (pin->flags[0])
    return set_err(GSK_ERR_INVALID_ARG,
                   "CSR structure invalid (row_ptr not monotone from 0 to nnz, or a column "
                   "index outside [0, n))");
  if (pin->flags[2]) return set_err(GSK_ERR_NONFINITE, "non-finite entry or row norm overflow");
  if (pin->flags[1]) return set_err(GSK_ERR_ZERO_ROW, "a row of A has zero Lp-norm");
  return GSK_OK;
}

int gsk_spmv(const gsk_matrix* A, const double* x, double* y, void* stream) {
  g_err.clear();
  Mat M;
  int rc = check_matrix(A, M);
  if (rc) return rc;
  if (!x || !y) return set_err(GSK_ERR_INVALID_ARG, "x or y is NULL");
  hipError_t e = launch_spmv(M, x, y, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_err(e, "spmv launch");
  return GSK_OK;
}

int gsk_stencil_from_csr(const gsk_csr* A, int32_t nx, int32_t ny, int32_t nz, double* coef,
                         void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  int rc = check_csr(A);
  if (rc) return rc;
  if (nx < 2 || ny < 2 || nz < 1 || (int64_t)nx * ny * nz != (int64_t)A->n)
    return set_err(GSK_ERR_INVALID_ARG, "grid %d x %d x %d does not match n = %d (need nx, ny "
                   ">= 2, nz >= 1)", (int)nx, (int)ny, (int)nz, (int)A->n);
  if (!coef) return set_err(GSK_ERR_INVALID_ARG, "coef is NULL");
  rc = check_ws(ws, ws_bytes, gsk::workspace_bytes(GSK_METHOD_GS, A->n, 0));
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace W = carve(ws, A->n);
  Csr C = to_csr(A);
  hipError_t e;
  if ((e = launch_clear_flags(W.flags, s)) != hipSuccess) return hip_err(e, "clear flags");
  if ((e = launch_validate(C, W.flags, s)) != hipSuccess) return hip_err(e, "validate");
  if ((e = launch_stencil_from_csr(C, nx, ny, nz, coef, W.flags, s)) != hipSuccess)
    return hip_err(e, "stencil_from_csr launch");
  Pinned* pin = pinned();
  if (!pin) return set_err(GSK_ERR_DEVICE, "pinned host buffer allocation failed");
  if ((e = hipMemcpyAsync(pin->flags, W.flags, 4 * sizeof(int), hipMemcpyDeviceToHost, s)) !=
      hipSuccess)
    return hip_err(e, "flag read-back");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_err(e, "stencil_from_csr");
  if (pin->flags[0])
    return set_err(GSK_ERR_INVALID_ARG,
                   "CSR structure invalid (row_ptr not monotone from 0 to nnz, or a column "
                   "index outside [0, n))");
  if (pin->flags[3])
    return set_err(GSK_ERR_INVALID_ARG,
                   "an entry is not a 5/7-point stencil position of its row, or repeats one");
  return GSK_OK;
}

int gsk_arnoldi(const gsk_matrix* A, const double* r0, int32_t m, double* V, int64_t ldv,
                double* H, int32_t* steps, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  Mat M;
  int rc = check_matrix(A, M);
  if (rc) return rc;
  if (m < 1 || m > GSK_MAX_RESTART)
    return set_err(GSK_ERR_INVALID_ARG, "m = %d must be in [1, %d]", (int)m, GSK_MAX_RESTART);
  if (!r0 || !V || !H || !steps) return set_err(GSK_ERR_INVALID_ARG, "NULL argument");
  if (ldv < M.n) return set_err(GSK_ERR_INVALID_ARG, "ldv < n");
  rc = check_ws(ws, ws_bytes, gsk::workspace_bytes(GSK_METHOD_ARNOLDI, M.n, m));
  if (rc) return rc;
  SolveResult r = arnoldi_run(M, r0, m, V, ldv, H, ws, 1e-16 * DBL_EPSILON,
                              static_cast<hipStream_t>(stream));
  if (r.code == -1)
    return set_err(GSK_ERR_INVALID_ARG, "invalid CSR structure or zero/non-finite r0");
  if (r.code) return set_err(GSK_ERR_DEVICE, "arnoldi: HIP failure (%s)",
                             hipGetErrorString(hipGetLastError()));
  *steps = r.sum.steps;
  return GSK_OK;
}

static int solve_common(int method, const gsk_matrix* A, const double* b, double* x,
                        int32_t m, double tol, const gsk_options* opt, gsk_info* info, void* ws,
                        size_t ws_bytes, void* stream) {
  g_err.clear();
  Mat M;
  int rc = check_matrix(A, M);
  if (rc) return rc;
  if (!b || !x) return set_err(GSK_ERR_INVALID_ARG, "b or x is NULL");
  const bool is_gmres = method != GSK_METHOD_BICGSTAB;
  if (is_gmres && (m < 1 || m > GSK_MAX_RESTART))
    return set_err(GSK_ERR_INVALID_ARG, "m = %d must be in [1, %d]", (int)m, GSK_MAX_RESTART);
  SolveParams prm;
  rc = params_from(opt, prm, tol);
  if (rc) return rc;
  rc = check_ws(ws, ws_bytes, gsk::workspace_bytes_for(M, method, m));
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  SolveResult r = method == GSK_METHOD_GMRES         ? gmres_solve(M, b, x, m, prm, ws, s)
                  : method == GSK_METHOD_GMRES_MIXED ? gmres_mixed_solve(M, b, x, m, prm, ws, s)
                                                     : bicgstab_solve(M, b, x, prm, ws, s);
  if (r.code == -1)
    return set_err(GSK_ERR_INVALID_ARG,
                   "CSR structure invalid (row_ptr not monotone from 0 to nnz, or a column "
                   "index outside [0, n))");
  if (r.code) return set_err(GSK_ERR_DEVICE, "solver: HIP failure (%s)",
                             hipGetErrorString(hipGetLastError()));
  fill_info(info, r.sum);
  return GSK_OK;
}

int gsk_gmres(const gsk_matrix* A, const double* b, double* x, int32_t m, double tol,
              const gsk_options* opt, gsk_info* info, void* ws, size_t ws_bytes, void* stream) {
  const Range range("gsk_gmres");
  return solve_common(GSK_METHOD_GMRES, A, b, x, m, tol, opt, info, ws, ws_bytes, stream);
}

int gsk_gmres_mixed(const gsk_matrix* A, const double* b, double* x, int32_t m, double tol,
                    const gsk_options* opt, gsk_info* info, void* ws, size_t ws_bytes,
                    void* stream) {
  const Range range("gsk_gmres_mixed");
  return solve_common(GSK_METHOD_GMRES_MIXED, A, b, x, m, tol, opt, info, ws, ws_bytes, stream);
}

int gsk_bicgstab(const gsk_matrix* A, const double* b, double* x, double tol,
                 const gsk_options* opt, gsk_info* info, void* ws, size_t ws_bytes,
                 void* stream) {
  const Range range("gsk_bicgstab");
  return solve_common(GSK_METHOD_BICGSTAB, A, b, x, 0, tol, opt, info, ws, ws_bytes, stream);
}

int gsk_bicgstab_noalloc(const gsk_matrix* A, const double* b, double* x, double tol,
                         const gsk_options* opt, gsk_info* info, void* stream) {
  g_err.clear();
  Mat M;
  int rc = check_matrix(A, M);
  if (rc) return rc;
  if (!b || !x) return set_err(GSK_ERR_INVALID_ARG, "b or x is NULL");
  SolveParams prm;
  rc = params_from(opt, prm, tol);
  if (rc) return rc;
  const size_t need = gsk::workspace_bytes(GSK_METHOD_BICGSTAB, M.n, 0);
  if (need > gsk::kNoAllocBytes)
    return set_err(GSK_ERR_WORKSPACE,
                   "a system of %d rows needs %zu bytes of scratch; the no-allocation entry "
                   "point holds %zu (use gsk_bicgstab with a workspace)",
                   (int)M.n, need, gsk::kNoAllocBytes);
  hipError_t e = hipSuccess;
  void* ptr = gsk::noalloc_scratch(&e);
  if (!ptr) return hip_err(e, "scratch address");
  hipStream_t s = static_cast<hipStream_t>(stream);
  SolveResult r = gsk::bicgstab_solve_noalloc(M, b, x, prm, ptr, s);
  if (r.code == -1)
    return set_err(GSK_ERR_INVALID_ARG,
                   "CSR structure invalid (row_ptr not monotone from 0 to nnz, or a column "
                   "index outside [0, n))");
  if (r.code) return set_err(GSK_ERR_DEVICE, "solver: HIP failure (%s)",
                             hipGetErrorString(hipGetLastError()));
  fill_info(info, r.sum);
  return GSK_OK;
}

size_t gsk_bicgstab_noalloc_max_bytes(void) { return gsk::kNoAllocBytes; }

}  // extern "C"
