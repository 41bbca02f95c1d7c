// Batched Bi-CGSTAB and the solve engine: many independent systems share every launch.
//
// Each system is one Bi-CGSTAB solve of section 2 (shadow residual r^ = r0, the stop test of
// section 2.2), exactly as in bicgstab.hip: the same kernels' arithmetic, the same tile
// partition of its rows, the same per-tile partials summed in the same order. A system
// therefore returns bit for bit the result it returns when solved alone with gsk_bicgstab,
// whatever else shares the batch.
//
// Layout. The engine owns a workspace with room for max_rows rows of vectors (r, r^, p x2,
// v x2, t) and max_systems control blocks. A system of n rows gets ceil(n / BS) consecutive
// tiles of that row space (first fit over free tiles); its matrix, b, x and stop weights stay
// in the caller's memory. A device list holds the tiles of the admitted systems (with each
// tile's system); a streaming launch has one workgroup per list entry (the grid rounded up
// to a few sizes, each with its own captured graph), so it costs work only for admitted
// systems; a finalize launch has one workgroup per system slot and sums that
// system's tile partials.
//
// A system may be submitted unscaled with a GS(p) stage (section 2, eq. (2)): the first chunk
// scales its rows into caller-provided outputs (with the arithmetic of gsk_gs_scale) and the
// solve then runs on the scaled system, so GS(p) and Bi-CGSTAB run in the same launches.
//
// Time. The host enqueues chunks: the GS launch (scales newly admitted systems that asked for
// it), the residual launch (starts newly admitted systems and verifies convergence claims),
// then check_every iterations. For a given grid size a chunk has fixed launch shapes and
// arguments, so it can be captured once in a HIP graph and replayed. Between
// chunks the host reads every slot's status and retires finished systems; new systems are
// admitted between chunks (continuous batching).
#include <map>
#include <vector>

#include "bicg_batch.hpp"

namespace gsk {

__global__ __launch_bounds__(64) void k_batch_init(BCtl* c, int maxit, double tol, double eps_b,
                                                   int has_w, int scale) {
  if (threadIdx.x != 0) return;
  c->sum.state = scale ? ST_SCALE : ST_INIT;
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
  c->first = 1;
  c->has_w = has_w;
  c->bad = 0;
  c->fp64 = 0;
  c->run_start = 0;
  c->tol = tol;
  c->eps_b = eps_b;
  c->ref = 0.0;
  c->rho = c->rho_old = c->alpha = c->omega = c->beta = c->rh_norm = 0.0;
  c->target = tol;
  c->last_rt = 1.0;
}

// Flat validity scan of one system's CSR structure (no indirect loads): row_ptr[0] == 0,
// non-decreasing, row_ptr[n] == nnz, every column index in [0, n). Sets BAD_CSR in *bad_bits.
__global__ __launch_bounds__(BS) void k_batch_validate(const int* __restrict__ rp,
                                                       const int* __restrict__ ci, int n,
                                                       int64_t nnz, int* bad_bits) {
  const int64_t stride = (int64_t)gridDim.x * BS;
  const int64_t gid = (int64_t)blockIdx.x * BS + threadIdx.x;
  bool bad = false;
  for (int64_t i = gid; i <= n; i += stride) {
    const int r = rp[i];
    if (i == 0 && r != 0) bad = true;
    if (i < n && r > rp[i + 1]) bad = true;
    if (i == n && (int64_t)r != nnz) bad = true;
  }
  for (int64_t k = gid; k < nnz; k += stride) {
    const int col = ci[k];
    if (col < 0 || col >= n) bad = true;
  }
  if (bad) atomicOr(bad_bits, BAD_CSR);
}

// G: GS(p) of the systems whose stage is pending (same arithmetic as k_gs_scale).
__global__ __launch_bounds__(BS) void k_batch_gs(BArgsB a) {
  __shared__ GsLds L;
  for_active_tiles(a, [&](int tile, int s) {
    const SysDesc d = a.sys[s];
    BCtl* c = a.ctl + s;
    if (c->sum.state != ST_SCALE || (c->bad & BAD_CSR)) return;
    prepare_tile(d, tile - d.tile_off, L, &c->bad);
  });
}

__global__ __launch_bounds__(64) void k_batch_fin_gs(BArgsB a) {
  const int s = blockIdx.x;
  if (threadIdx.x != 0 || a.sys[s].ntiles == 0) return;
  BCtl* c = a.ctl + s;
  if (c->sum.state != ST_SCALE) return;
  c->sum.state = ST_INIT;   // a GS error (c->bad) is reported by the residual stage
}

// R: r = b - A x, r^ = r for systems starting, verifying or finishing; ||r||^2, ||W r||^2.
__global__ __launch_bounds__(BS) void k_batch_residual(BArgsB a) {
  __shared__ TileLds L;
  __shared__ double red[NC_MAX * WAVES];
  for_active_tiles(a, [&](int tile, int s) {
    const BCtl* c = a.ctl + s;
    const int st = c->sum.state;
    if (st != ST_INIT && st != ST_VERIFY && st != ST_FINAL) return;
    if (c->bad) return;
    bicg64_residual_tile(a, tile, s, st, L, red);
  });
}

__global__ __launch_bounds__(BS) void k_batch_fin_residual(BArgsB a) {
  const int s = blockIdx.x;
  const SysDesc d = a.sys[s];
  if (d.ntiles == 0) return;
  BCtl* c = a.ctl + s;
  const int st = c->sum.state;
  if (st != ST_INIT && st != ST_VERIFY && st != ST_FINAL) return;
  if (c->bad) {
    if (threadIdx.x == 0) {
      c->sum.state = ST_DONE;
      c->sum.status = bad_status(c->bad);
    }
    return;
  }
  __shared__ double out[8];
  small_sums_strided<2>(a.partials + d.tile_off, d.ntiles, a.max_tiles, out);
  if (threadIdx.x != 0) return;
  const double nr = sqrt(out[0]);
  const double nwr = d.W ? sqrt(out[1]) : nr;
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
}

// P: new p, v = A p; partials (r^, v), ||v||^2.
template <int RV>
__global__ __launch_bounds__(BS) void k_batch_p(BArgsB a) {
  __shared__ UnitLds U;
  TileLds& L = U.csr;
  __shared__ double red[NC_MAX * WAVES];
  if constexpr (RV == 1) {
    for_active_tiles(a, [&](int tile, int s) {
      const SysDesc d = a.sys[s];
      BCtl* c = a.ctl + s;
      if (c->sum.state != ST_RUNNING) return;
      const int q = a.par;
      const int64_t o = d.row_off;
      const GatherPB G{a.r + o, a.p[q] + o, a.v[q] + o, c->beta, c->omega, c->first};
      const int row0 = (tile - d.tile_off) * BS;
      const int nrows = min(BS, d.n - row0);
      const int t = threadIdx.x;
      const double y = sys_tile(d, row0, nrows, G, L);
      double acc[2] = {0.0, 0.0};
      if (t < nrows) {
        const int row = row0 + t;
        a.p[q ^ 1][o + row] = G(row);
        a.v[q ^ 1][o + row] = y;
        acc[0] = a.rh[o + row] * y;
        acc[1] = y * y;
      }
      block_partials<2>(acc, 2, a.partials, a.max_tiles, tile, red);
    });
  } else {
    // two tiles per workgroup
    for_active_units(a, [&](int unit, int s) {
      if (a.ctl[s].sum.state != ST_RUNNING) return;
      bicg64_p_unit2(a, unit, s, U, red);
    });
  }
}

__global__ __launch_bounds__(BS) void k_batch_fin_p(BArgsB a) {
  const int s = blockIdx.x;
  const SysDesc d = a.sys[s];
  if (d.ntiles == 0) return;
  BCtl* c = a.ctl + s;
  if (c->sum.state != ST_RUNNING) return;
  __shared__ double out[8];
  small_sums_strided<2>(a.partials + d.tile_off, d.ntiles, a.max_tiles, out);
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

// S: t = A s with s = r - alpha v; partials (t,s), (t,t), ||s||^2, ||W s||^2.
template <int RV>
__global__ __launch_bounds__(BS) void k_batch_s(BArgsB a) {
  __shared__ UnitLds U;
  TileLds& L = U.csr;
  __shared__ double red[NC_MAX * WAVES];
  if constexpr (RV == 1) {
    for_active_tiles(a, [&](int tile, int s) {
      const SysDesc d = a.sys[s];
      BCtl* c = a.ctl + s;
      if (c->sum.state != ST_RUNNING) return;
      const int64_t o = d.row_off;
      const GatherSB G{a.r + o, a.v[a.par ^ 1] + o, c->alpha};
      const int row0 = (tile - d.tile_off) * BS;
      const int nrows = min(BS, d.n - row0);
      const int t = threadIdx.x;
      const double y = sys_tile(d, row0, nrows, G, L);
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      if (t < nrows) {
        const int row = row0 + t;
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
      block_partials<4>(acc, 4, a.partials, a.max_tiles, tile, red);
    });
  } else {
    for_active_units(a, [&](int unit, int s) {
      if (a.ctl[s].sum.state != ST_RUNNING) return;
      bicg64_s_unit2(a, unit, s, U, red);
    });
  }
}

__global__ __launch_bounds__(BS) void k_batch_fin_s(BArgsB a) {
  const int s = blockIdx.x;
  const SysDesc d = a.sys[s];
  if (d.ntiles == 0) return;
  BCtl* c = a.ctl + s;
  if (c->sum.state != ST_RUNNING) return;
  __shared__ double out[8];
  small_sums_strided<4>(a.partials + d.tile_off, d.ntiles, a.max_tiles, out);
  if (threadIdx.x != 0) return;
  c->sum.iters += 1;
  const double sn = sqrt(out[2]);
  const double est = (d.W ? sqrt(out[3]) : sn) / c->ref;
  c->sum.relres_rec = est;
  if (est < c->tol) {
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

// U: x += alpha p + omega s, r = s - omega t; partials (r^, r), ||r||^2, ||W r||^2.
// After a half-step exit only x += alpha p is done.
__global__ __launch_bounds__(BS) void k_batch_u(BArgsB a) {
  __shared__ double red[NC_MAX * WAVES];
  for_active_tiles(a, [&](int tile, int s) {
    const int st = a.ctl[s].sum.state;
    if (st != ST_RUNNING && st != ST_HALF) return;
    bicg64_u_tile(a, tile, s, st, red);
  });
}

__global__ __launch_bounds__(BS) void k_batch_fin_u(BArgsB a) {
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
  small_sums_strided<3>(a.partials + d.tile_off, d.ntiles, a.max_tiles, out);
  if (threadIdx.x != 0) return;
  const double rn = sqrt(out[1]);
  const double est = (d.W ? sqrt(out[2]) : rn) / c->ref;
  c->sum.relres_rec = est;
  if (est < c->tol || c->sum.iters >= c->maxit) {
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

// Measurement: the algorithmic bytes of the launch of class kc that ran just before (per
// system at that stage, the figures of the kernel-class table in gsk.h), into ps->bytes[slot].
// Runs between that launch and its finalize, so every system is in the state the launch saw.
__global__ __launch_bounds__(BS) void k_batch_probe_bytes(BArgsB a, int max_sys, int kc,
                                                          int cls, int slot, ProbeSlots* ps) {
  __shared__ double red[NC_MAX * WAVES];
  double acc[1] = {0.0};
  for (int s = threadIdx.x; s < max_sys; s += BS) {
    const SysDesc d = a.sys[s];
    if (d.ntiles == 0 || d.cls != cls) continue;
    const BCtl* c = a.ctl + s;
    const int st = c->sum.state;
    const double n = (double)d.n;
    if (kc == KC_BATCH_U) {
      if (st == ST_RUNNING) acc[0] += (d.W ? 72.0 : 64.0) * n;
      if (st == ST_HALF) acc[0] += 24.0 * n;
      continue;
    }
    if (st != ST_RUNNING) continue;
    // matrix term (a running system's CSR structure has been validated)
    const double M = d.kind == MAT_STENCIL ? 8.0 * (d.nz > 1 ? 7 : 5) * n
                                           : 12.0 * (double)d.rp[d.n] + 4.0 * (n + 1.0);
    if (kc == KC_BATCH_P) acc[0] += M + (c->first ? 32.0 : 48.0) * n;
    if (kc == KC_BATCH_S) acc[0] += M + (d.W ? 32.0 : 24.0) * n;
  }
  block_partials<1>(acc, 1, ps->bytes, 0, slot, red);
}

// ---------------------------------------------------------------------------------------
// Host side: the engine.
// ---------------------------------------------------------------------------------------
constexpr int kBatchVectors = 7;

struct EngineLayout {
  size_t sys, tiles, probe, ctl, sums, partials, vecs, total;
};

static bool per_class(const EngineConfig& cfg) {
  return cfg.method == 0 && !cfg.mixed &&
         (cfg.class_shape[0] | cfg.class_shape[1] | cfg.class_shape[2]) != 0;
}

static int classes_of(const EngineConfig& cfg) { return per_class(cfg) ? kClassCount : 1; }

static int units_of(const EngineConfig& cfg) {
  if (cfg.mixed || per_class(cfg)) return 2;
  return cfg.method == 0 && cfg.units == 2 ? 2 : 1;   // FP64 Bi-CGSTAB may take two
}

// Size class of a system in an engine with per-class shapes.
static int class_of(const Mat& A) {
  if (A.kind != MAT_STENCIL || A.nz <= 1) return kClass2D;
  return A.n < kClassLargeRows ? kClass3DSmall : kClass3DLarge;
}

// Workspace carve-up. Bi-CGSTAB: system table, unit lists (per size class: units, slots;
// then the classes' counts), control blocks, partials (4 per tile), the 7 vectors. GMRES: system table, unit list, control blocks, status copies,
// partials (max(m+1, 3) columns per tile and one more for C), basis (m+1 columns) and w, in
// FP64 or FP32.
static EngineLayout engine_layout(const EngineConfig& cfg) {
  const int64_t max_tiles = (cfg.max_rows + BS - 1) / BS;
  const int64_t grid_tiles = (max_tiles + 7) / 8 * 8;
  const size_t ns = (size_t)cfg.max_sys;
  EngineLayout L;
  size_t off = 0;
  L.sys = off;
  off += align256(sizeof(SysDesc) * ns);
  L.tiles = off;
  off += align256(sizeof(int) * (size_t)classes_of(cfg) * (2 * (size_t)grid_tiles + 1));
  L.probe = off;
  off += align256(sizeof(ProbeSlots));
  L.ctl = off;
  if (cfg.method == 1) {
    off += align256(sizeof(Ctl) * ns);
    L.sums = off;
    off += align256(sizeof(Summary) * ns);
    L.partials = off;
    off += align256(sizeof(double) * (size_t)gmres_partial_cols(cfg.m) * (size_t)grid_tiles);
    L.vecs = off;
    const size_t tb = cfg.mixed ? sizeof(float) : sizeof(double);
    off += align256(tb * (size_t)grid_tiles * BS * (size_t)(cfg.m + 1));
    off += align256(tb * (size_t)grid_tiles * BS);
  } else {
    off += align256(sizeof(BCtl) * ns);
    L.sums = off;
    L.partials = off;
    off += align256(sizeof(double) * 4 * (size_t)grid_tiles);
    L.vecs = off;
    const size_t rows = (size_t)grid_tiles * BS;
    if (cfg.mixed)   // FP32 vectors, then the FP64 continuation's vectors and the saved x
      off += (size_t)kBatchVectors * align256(sizeof(float) * rows) +
             (size_t)(kBatchVectors + 1) * align256(sizeof(double) * rows);
    else
      off += (size_t)kBatchVectors * align256(sizeof(double) * rows);
  }
  L.total = off;
  return L;
}

size_t engine_workspace_bytes(const EngineConfig& cfg) {
  if (cfg.max_rows < 1 || cfg.max_sys < 1) return 0;
  if (cfg.method == 1 && (cfg.m < 1 || cfg.m > MMAX)) return 0;
  return engine_layout(cfg).total;
}

struct Engine {
  hipStream_t s = nullptr;
  int64_t max_rows = 0;
  int max_sys = 0, max_tiles = 0, grid_tiles = 0, check_every = 8;
  bool use_graph = false;
  int method = 0;                  // 0 Bi-CGSTAB, 1 GMRES(m)
  int m = 0;
  bool mixed = false;
  int rv = 1;                      // tiles per unit
  int max_units = 0;
  int nclass = 1;                  // size classes, each with its own unit list and launches
  int shape[kClassCount] = {kShapeTile, kShapeTile, kShapeTile};
  bool column = true;              // GMRES basis fits one buffer descriptor
  BArgsB args{};
  GArgs gargs{};
  MArgs margs{};
  SysDesc* d_sys = nullptr;        // device system table and unit list (any method)
  int* d_list = nullptr;
  ProbeSlots* d_probe = nullptr;   // measurement slots (FP64 Bi-CGSTAB engine)
  long long probe_chunks = 0;      // chunks run while a batch kernel class is probed
  bool probe_pending = false;      // timed launches wait for their collection at the next poll
  // host state
  std::vector<SysDesc> h_sys;
  std::vector<int64_t> tags;
  std::vector<char> active;
  std::vector<int> tile_sys;       // slot of every tile, -1 if free
  std::map<int, int> free_tiles;   // start -> length
  bool dirty = true;
  int64_t launched = 0;
  // pinned staging and status
  SysDesc* p_sys = nullptr;
  int* p_tiles = nullptr;
  BCtl* p_ctl = nullptr;
  Summary* p_sums = nullptr;
  hipEvent_t ev_upload = nullptr, ev_chunk = nullptr;
  bool upload_pending = false, chunk_pending = false;
  int n_listed[kClassCount] = {0, 0, 0};     // entries of each class's device unit list
  std::map<std::vector<int>, hipGraphExec_t> graphs;   // captured chunk per grid sizes
};

static const Summary& status_of(const Engine& e, int slot) {
  return e.method == 1 ? e.p_sums[slot] : e.p_ctl[slot].sum;
}

// Streaming grid for a list of n tiles: n rounded up to a multiple of 8 (the XCD mapping of
// logical_block needs it) and, from 32 on, to two significant bits (4..7 times a power of two),
// so that the grid, and the captured graph that holds it, changes only when the list has grown
// or shrunk by about a quarter; the surplus workgroups exit at once.
static int stream_grid(int n) {
  int g = n < 8 ? 8 : (n + 7) / 8 * 8;
  int top = 1;
  while (top * 2 <= g) top *= 2;
  if (top >= 32) {
    const int step = top / 4;
    g = (g + step - 1) / step * step;
  }
  return g;
}

static bool alloc_tiles(Engine& e, int need, int& start) {
  for (auto it = e.free_tiles.begin(); it != e.free_tiles.end(); ++it) {
    if (it->second >= need) {
      start = it->first;
      const int rest = it->second - need;
      e.free_tiles.erase(it);
      if (rest > 0) e.free_tiles[start + need] = rest;
      return true;
    }
  }
  return false;
}

static void free_tiles_range(Engine& e, int start, int len) {
  auto it = e.free_tiles.emplace(start, len).first;
  auto next = std::next(it);
  if (next != e.free_tiles.end() && it->first + it->second == next->first) {
    it->second += next->second;
    e.free_tiles.erase(next);
  }
  if (it != e.free_tiles.begin()) {
    auto prev = std::prev(it);
    if (prev->first + prev->second == it->first) {
      prev->second += it->second;
      e.free_tiles.erase(it);
    }
  }
}

int engine_create(void* ws, size_t ws_bytes, const EngineConfig& cfg, hipStream_t s,
                  Engine** out) {
  if (cfg.max_rows < 1 || cfg.max_sys < 1) return -1;
  if (cfg.method == 1 && (cfg.m < 1 || cfg.m > MMAX)) return -1;
  const EngineLayout L = engine_layout(cfg);
  if (ws_bytes < L.total) return -4;
  if (cfg.use_graph && (s == nullptr || (cfg.method == 0 && (cfg.check_every & 1)))) return -1;
  Engine* e = new Engine();
  e->s = s;
  e->max_rows = cfg.max_rows;
  e->max_sys = cfg.max_sys;
  e->max_tiles = (int)((cfg.max_rows + BS - 1) / BS);
  e->grid_tiles = (e->max_tiles + 7) / 8 * 8;
  e->check_every = cfg.check_every;
  e->use_graph = cfg.use_graph;
  e->method = cfg.method;
  e->m = cfg.m;
  e->mixed = cfg.mixed;
  e->rv = units_of(cfg);
  e->max_units = e->grid_tiles / e->rv;
  e->nclass = classes_of(cfg);
  if (per_class(cfg)) {
    const int dflt = cfg.units == 2 ? kShapePair : kShapeTile;
    for (int c = 0; c < kClassCount; ++c)
      e->shape[c] = cfg.class_shape[c] ? cfg.class_shape[c] : dflt;
  } else {
    e->shape[0] = e->rv == 2 ? kShapePair : kShapeTile;
  }
  const int max_sys = cfg.max_sys;
  char* base = static_cast<char*>(ws);
  if (e->method == 1) {
    GArgs& g = e->gargs;
    g.sys = reinterpret_cast<const SysDesc*>(base + L.sys);
    g.act = reinterpret_cast<const int*>(base + L.tiles);
    g.n_act = g.act + 2 * (size_t)e->max_units;
    g.ctl = reinterpret_cast<Ctl*>(base + L.ctl);
    g.sums = reinterpret_cast<Summary*>(base + L.sums);
    g.partials = reinterpret_cast<double*>(base + L.partials);
    g.pstride = e->grid_tiles;
    g.ccol = gmres_partial_cols(cfg.m) - 1;
    g.max_units = e->max_units;
    g.ldv = (size_t)e->grid_tiles * BS;
    const size_t tb = e->mixed ? sizeof(float) : sizeof(double);
    g.V = base + L.vecs;
    g.w = base + L.vecs + align256(tb * g.ldv * (size_t)(cfg.m + 1));
    g.zero = 0.0;
    g.mixed = e->mixed ? 1 : 0;
    e->column = e->mixed ? fits_buffer<float>(g.ldv, cfg.m + 1)
                         : fits_buffer<double>(g.ldv, cfg.m + 1);
  } else if (e->mixed) {
    MArgs& a = e->margs;
    a.sys = reinterpret_cast<const SysDesc*>(base + L.sys);
    a.act = reinterpret_cast<const int*>(base + L.tiles);
    a.n_act = a.act + 2 * (size_t)e->max_units;
    a.ctl = reinterpret_cast<BCtl*>(base + L.ctl);
    a.partials = reinterpret_cast<double*>(base + L.partials);
    a.pstride = e->grid_tiles;
    a.max_units = e->max_units;
    const size_t rows = (size_t)e->grid_tiles * BS;
    const size_t vbf = align256(sizeof(float) * rows), vbd = align256(sizeof(double) * rows);
    float* v[kBatchVectors];
    double* w[kBatchVectors + 1];
    for (int i = 0; i < kBatchVectors; ++i)
      v[i] = reinterpret_cast<float*>(base + L.vecs + i * vbf);
    for (int i = 0; i <= kBatchVectors; ++i)
      w[i] = reinterpret_cast<double*>(base + L.vecs + kBatchVectors * vbf + i * vbd);
    a.r = v[0];
    a.rh = v[1];
    a.p[0] = v[2];
    a.p[1] = v[3];
    a.v[0] = v[4];
    a.v[1] = v[5];
    a.t = v[6];
    a.r64 = w[0];
    a.rh64 = w[1];
    a.p64[0] = w[2];
    a.p64[1] = w[3];
    a.v64[0] = w[4];
    a.v64[1] = w[5];
    a.t64 = w[6];
    a.xprev = w[7];
    a.delta = cfg.delta;
    a.run_cap = cfg.run_cap;
    a.par = 0;
    e->args.ctl = a.ctl;   // status read-back
  } else {
    BArgsB& a = e->args;
    a.sys = reinterpret_cast<const SysDesc*>(base + L.sys);
    a.act = reinterpret_cast<const int*>(base + L.tiles);
    a.ctl = reinterpret_cast<BCtl*>(base + L.ctl);
    a.partials = reinterpret_cast<double*>(base + L.partials);
    a.max_tiles = e->grid_tiles;
    a.max_units = e->max_units;
    a.rv = e->rv;
    a.split = 0;
    a.n_act = a.act + 2 * (size_t)e->max_units;
    const size_t vb = align256(sizeof(double) * (size_t)e->grid_tiles * BS);
    double* v[kBatchVectors];
    for (int i = 0; i < kBatchVectors; ++i)
      v[i] = reinterpret_cast<double*>(base + L.vecs + i * vb);
    a.r = v[0];
    a.rh = v[1];
    a.p[0] = v[2];
    a.p[1] = v[3];
    a.v[0] = v[4];
    a.v[1] = v[5];
    a.t = v[6];
    a.par = 0;
  }
  e->d_sys = reinterpret_cast<SysDesc*>(base + L.sys);
  e->d_list = reinterpret_cast<int*>(base + L.tiles);
  e->d_probe = reinterpret_cast<ProbeSlots*>(base + L.probe);
  e->h_sys.assign(max_sys, SysDesc{});
  e->tags.assign(max_sys, 0);
  e->active.assign(max_sys, 0);
  e->tile_sys.assign(e->grid_tiles, -1);
  e->free_tiles[0] = e->max_tiles;
  bool ok = hipHostMalloc((void**)&e->p_sys, sizeof(SysDesc) * max_sys, hipHostMallocDefault) ==
                hipSuccess &&
            hipHostMalloc((void**)&e->p_tiles,
                          sizeof(int) * (size_t)e->nclass * (2 * (size_t)e->max_units + 1),
                          hipHostMallocDefault) == hipSuccess &&
            hipEventCreateWithFlags(&e->ev_upload, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&e->ev_chunk, hipEventDisableTiming) == hipSuccess;
  if (ok && e->method == 1)
    ok = hipHostMalloc((void**)&e->p_sums, sizeof(Summary) * max_sys, hipHostMallocDefault) ==
         hipSuccess;
  if (ok && e->method == 0)   // FP64 and mixed Bi-CGSTAB share the control block layout
    ok = hipHostMalloc((void**)&e->p_ctl, sizeof(BCtl) * max_sys, hipHostMallocDefault) ==
         hipSuccess;
  if (!ok) {
    engine_destroy(e);
    return -5;
  }
  *out = e;
  return 0;
}

void engine_destroy(Engine* e) {
  if (!e) return;
  if (e->s) (void)hipStreamSynchronize(e->s);
  for (auto& kv : e->graphs) (void)hipGraphExecDestroy(kv.second);
  if (e->ev_upload) (void)hipEventDestroy(e->ev_upload);
  if (e->ev_chunk) (void)hipEventDestroy(e->ev_chunk);
  if (e->p_sys) (void)hipHostFree(e->p_sys);
  if (e->p_tiles) (void)hipHostFree(e->p_tiles);
  if (e->p_ctl) (void)hipHostFree(e->p_ctl);
  if (e->p_sums) (void)hipHostFree(e->p_sums);
  delete e;
}

// The pinned staging buffers may be rewritten only after the previous upload has run.
static int wait_upload(Engine& e) {
  if (e.upload_pending) {
    if (hipEventSynchronize(e.ev_upload) != hipSuccess) return -5;
    e.upload_pending = false;
  }
  return 0;
}

int engine_submit(Engine* e, const Mat& A, const double* b, double* x, const SolveParams& prm,
                  int64_t tag, const GsStage* gs) {
  int slot = -1;
  for (int i = 0; i < e->max_sys; ++i) {
    if (e->active[i] && e->tags[i] == tag) return -6;   // the tag is still in flight
    if (slot < 0 && !e->active[i]) slot = i;
  }
  if (slot < 0) return 1;   // no free slot
  if (e->mixed && (!gs || !gs->mat32)) return -1;
  const int need = (A.n + BS - 1) / BS;
  const int held = (need + e->rv - 1) / e->rv * e->rv;   // whole units
  int start = 0;
  if (!alloc_tiles(*e, held, start)) return 1;   // no room
  SysDesc d{};
  d.n = A.n;
  d.kind = A.kind;
  d.nx = A.nx;
  d.ny = A.ny;
  d.nz = A.nz;
  d.tile_off = start;
  d.ntiles = need;
  d.unit_off = start / e->rv;
  d.nunits = held / e->rv;
  d.cls = e->nclass > 1 ? class_of(A) : 0;
  d.row_off = (int64_t)start * BS;
  d.rp = A.csr.rp;
  d.ci = A.csr.ci;
  d.val = A.csr.val;
  d.coef = A.coef;
  d.b = b;
  d.x = x;
  d.W = prm.weights;
  d.gs_p = 0;
  d.mat32 = nullptr;
  d.ldp32 = 0;
  if (gs && gs->p > 0) {   // the solve reads the GS outputs
    d.gs_p = gs->p;
    d.gs_val = A.kind == MAT_STENCIL ? A.coef : A.csr.val;
    d.gs_b = b;
    if (A.kind == MAT_STENCIL) d.coef = gs->val_out;
    else d.val = gs->val_out;
    d.b = gs->b_out;
    d.W = gs->weight_out;
  }
  if (e->mixed) {
    d.mat32 = gs->mat32;
    d.ldp32 = gs->ldp32;
  }
  const bool prepare = d.gs_p > 0 || d.mat32 != nullptr;
  e->h_sys[slot] = d;
  e->tags[slot] = tag;
  e->active[slot] = 1;
  for (int t = 0; t < held; ++t) e->tile_sys[start + t] = slot;
  e->dirty = true;
  int* bad = nullptr;
  if (e->method == 1) {
    Ctl* c = e->gargs.ctl + slot;
    bad = &c->bad;
    if (launch_gmres_init(c, prm.maxit, e->m, prm.tol, prm.eps_b, d.W ? 1 : 0, prepare ? 1 : 0,
                          e->s) != hipSuccess)
      return -5;
  } else {
    BCtl* c = e->args.ctl + slot;
    bad = &c->bad;
    hipLaunchKernelGGL(k_batch_init, dim3(1), dim3(64), 0, e->s, c, prm.maxit, prm.tol,
                       prm.eps_b, d.W ? 1 : 0, prepare ? 1 : 0);
  }
  if (A.kind == MAT_CSR) {
    int64_t blocks = ((int64_t)A.csr.nnz + A.n + BS) / BS;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_batch_validate, dim3((unsigned)blocks), dim3(BS), 0, e->s, A.csr.rp,
                       A.csr.ci, A.n, A.csr.nnz, bad);
  }
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

static int upload(Engine& e) {
  if (!e.dirty) return 0;
  if (wait_upload(e)) return -5;
  for (int i = 0; i < e.max_sys; ++i) {
    e.p_sys[i] = e.h_sys[i];
    if (!e.active[i]) e.p_sys[i].ntiles = 0;
  }
  // the units of every admitted system, in row-space order (a system's units are
  // consecutive, so adjacent list entries are adjacent rows of one system), each in its size
  // class's list; only the listed entries and the counts are copied, so a large engine costs
  // no more than a small one
  const size_t mu = (size_t)e.max_units;
  int n[kClassCount] = {0, 0, 0};
  for (int t = 0; t < e.grid_tiles;) {
    const int s = e.tile_sys[t];
    if (s < 0) {
      auto it = e.free_tiles.find(t);   // skip a free range in one step
      t += it != e.free_tiles.end() ? it->second : e.rv;
      continue;
    }
    const SysDesc& d = e.h_sys[s];
    int* list = e.p_tiles + (size_t)d.cls * 2 * mu;
    for (int u = 0; u < d.nunits; ++u) {
      list[n[d.cls]] = d.unit_off + u;
      list[mu + n[d.cls]] = s;
      ++n[d.cls];
    }
    t = d.tile_off + d.nunits * e.rv;
  }
  int* counts = e.p_tiles + (size_t)e.nclass * 2 * mu;
  bool ok = hipMemcpyAsync(e.d_sys, e.p_sys, sizeof(SysDesc) * e.max_sys,
                           hipMemcpyHostToDevice, e.s) == hipSuccess;
  for (int c = 0; c < e.nclass; ++c) {
    counts[c] = n[c];
    e.n_listed[c] = n[c];
    const size_t base = (size_t)c * 2 * mu;
    if (n[c] > 0)
      ok = ok &&
           hipMemcpyAsync(e.d_list + base, e.p_tiles + base, sizeof(int) * (size_t)n[c],
                          hipMemcpyHostToDevice, e.s) == hipSuccess &&
           hipMemcpyAsync(e.d_list + base + mu, e.p_tiles + base + mu,
                          sizeof(int) * (size_t)n[c], hipMemcpyHostToDevice, e.s) == hipSuccess;
  }
  ok = ok &&
       hipMemcpyAsync(e.d_list + (size_t)e.nclass * 2 * mu, counts, sizeof(int) * e.nclass,
                      hipMemcpyHostToDevice, e.s) == hipSuccess &&
       hipEventRecord(e.ev_upload, e.s) == hipSuccess;
  if (!ok) return -5;
  e.upload_pending = true;
  e.dirty = false;
  return 0;
}

// Launch of a streaming kernel of class kc over the systems of size class cls; in a sampled
// chunk (probed == kc) it carries a pair of timing events and is followed by the launch that
// records its algorithmic bytes.
template <class F>
static void launch_stream(Engine& e, F kernel, int kc, int probed, dim3 grid, const BArgsB& a,
                          int cls) {
  const int slot = probed == kc ? probe_slot_all(kc) : -1;
  launch_probed(kernel, grid, e.s, slot, a);
  if (slot >= 0)
    hipLaunchKernelGGL(k_batch_probe_bytes, dim3(1), dim3(BS), 0, e.s, a, e.max_sys, kc, cls,
                       slot, e.d_probe);
}

// Non-temporal policy of a GMRES chunk: the admitted systems' cycle working set (m + 2
// vectors of their rows, FP64 or FP32) exceeds the 256 MB last-level cache, so it streams from
// HBM once per launch whatever the policy.
static int gmres_streams(const Engine& e) {
  if (e.method != 1) return 0;
  const double rows = (double)e.n_listed[0] * e.rv * BS;
  return (double)(e.m + 2) * rows * (e.mixed ? 4.0 : 8.0) > kStreamBytes ? 1 : 0;
}

// Streaming grid of each size class's unit list (0: the class has no systems), then the GMRES
// load policy: what a captured chunk depends on.
static std::vector<int> class_grids(const Engine& e) {
  std::vector<int> g(e.nclass + 1, 0);
  for (int c = 0; c < e.nclass; ++c)
    g[c] = e.n_listed[c] > 0 || e.nclass == 1 ? stream_grid(e.n_listed[c]) : 0;
  g[e.nclass] = gmres_streams(e);
  return g;
}

static void enqueue_chunk(Engine& e, int k, int64_t first_iter, const std::vector<int>& grids,
                          int probed = 0) {
  if (e.method == 1) {
    (void)launch_gmres_chunk(e.gargs, e.m, grids[0], e.max_sys, e.column, grids[1] != 0, e.s);
    return;
  }
  if (e.mixed) {
    (void)launch_bicg_mixed_chunk(e.margs, k, first_iter, grids[0], e.max_sys, e.s);
    return;
  }
  // each class's launches read its own unit list; with units of two tiles, per-tile launches
  // (split) take a unit with two workgroups
  const size_t mu = (size_t)e.max_units;
  const dim3 gs(e.max_sys), block(BS);
  BArgsB ac[kClassCount];
  dim3 gu[kClassCount], gt[kClassCount];
  for (int c = 0; c < e.nclass; ++c) {
    ac[c] = e.args;
    ac[c].act = e.d_list + (size_t)c * 2 * mu;
    ac[c].n_act = e.d_list + (size_t)e.nclass * 2 * mu + c;
    gu[c] = dim3(grids[c]);
    gt[c] = dim3(grids[c] * (e.nclass > 1 ? e.rv : 1));
  }
  auto each = [&](auto body) {
    for (int c = 0; c < e.nclass; ++c)
      if (grids[c] > 0) body(c);
  };
  // per-tile launches: split in an engine with size classes (units of two tiles), otherwise
  // one workgroup per unit as before
  auto tiled = [&](int c) {
    BArgsB a = ac[c];
    a.split = e.nclass > 1 ? 1 : 0;
    return a;
  };
  each([&](int c) { hipLaunchKernelGGL(k_batch_gs, gt[c], block, 0, e.s, tiled(c)); });
  hipLaunchKernelGGL(k_batch_fin_gs, gs, dim3(64), 0, e.s, e.args);
  each([&](int c) { hipLaunchKernelGGL(k_batch_residual, gt[c], block, 0, e.s, tiled(c)); });
  hipLaunchKernelGGL(k_batch_fin_residual, gs, block, 0, e.s, e.args);
  for (int it = 0; it < k; ++it) {
    const int par = (int)((first_iter + it) & 1);
    for (int c = 0; c < e.nclass; ++c) ac[c].par = par;
    BArgsB fa = e.args;
    fa.par = par;
    each([&](int c) {
      if (e.shape[c] == kShapeTile) {
        BArgsB a = tiled(c);
        a.par = par;
        launch_stream(e, k_batch_p<1>, KC_BATCH_P, probed, gt[c], a, c);
      } else {
        launch_stream(e, k_batch_p<2>, KC_BATCH_P, probed, gu[c], ac[c], c);
      }
    });
    hipLaunchKernelGGL(k_batch_fin_p, gs, block, 0, e.s, fa);
    each([&](int c) {
      if (e.shape[c] == kShapeTile) {
        BArgsB a = tiled(c);
        a.par = par;
        launch_stream(e, k_batch_s<1>, KC_BATCH_S, probed, gt[c], a, c);
      } else {
        launch_stream(e, k_batch_s<2>, KC_BATCH_S, probed, gu[c], ac[c], c);
      }
    });
    hipLaunchKernelGGL(k_batch_fin_s, gs, block, 0, e.s, fa);
    each([&](int c) {
      if (e.shape[c] == kShapePair) {
        launch_stream(e, k_batch_u, KC_BATCH_U, probed, gu[c], ac[c], c);
      } else {
        BArgsB a = tiled(c);
        a.par = par;
        launch_stream(e, k_batch_u, KC_BATCH_U, probed, gt[c], a, c);
      }
    });
    hipLaunchKernelGGL(k_batch_fin_u, gs, block, 0, e.s, fa);
  }
}

int engine_run(Engine* e, int chunks) {
  if (upload(*e)) return -5;
  const int k = e->check_every;
  const std::vector<int> grid = class_grids(*e);
  hipGraphExec_t exec = nullptr;
  if (e->use_graph) {
    // Every Bi-CGSTAB chunk starts at an even iteration (k is even) and every GMRES chunk at
    // the start of a cycle, so one captured chunk per set of grid sizes serves all; the chunk
    // reads the unit lists and control blocks from device memory.
    auto it = e->graphs.find(grid);
    if (it != e->graphs.end()) {
      exec = it->second;
    } else {
      hipGraph_t g = nullptr;
      if (hipStreamBeginCapture(e->s, hipStreamCaptureModeThreadLocal) != hipSuccess) return -5;
      enqueue_chunk(*e, k, 0, grid);
      if (hipStreamEndCapture(e->s, &g) != hipSuccess) return -5;
      const hipError_t r = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (r != hipSuccess) return -5;
      e->graphs[grid] = exec;
    }
  }
  // measurement: while a batch kernel class is probed, every probe_every-th chunk is enqueued
  // without its graph, with that class's launches timed
  int probe_cls = 0, every = 0;
  if (e->method == 0 && !e->mixed) {
    for (int kc : {(int)KC_BATCH_P, (int)KC_BATCH_S, (int)KC_BATCH_U})
      if ((every = probe_every(kc)) > 0) {
        probe_cls = kc;
        break;
      }
  }
  for (int c = 0; c < chunks; ++c) {
    const bool sampled = probe_cls && (e->probe_chunks++ % every) == 0;
    if (sampled) {
      if (!e->probe_pending) probe_solve_begin();
      e->probe_pending = true;
      enqueue_chunk(*e, k, e->launched, grid, probe_cls);
    } else if (exec) {
      if (hipGraphLaunch(exec, e->s) != hipSuccess) return -5;
    } else {
      enqueue_chunk(*e, k, e->launched, grid);
    }
    e->launched += k;
  }
  if (hipGetLastError() != hipSuccess) return -5;
  const hipError_t cp =
      e->method == 1
          ? hipMemcpyAsync(e->p_sums, e->gargs.sums, sizeof(Summary) * e->max_sys,
                           hipMemcpyDeviceToHost, e->s)
          : hipMemcpyAsync(e->p_ctl, e->args.ctl, sizeof(BCtl) * e->max_sys,
                           hipMemcpyDeviceToHost, e->s);
  if (cp != hipSuccess || hipEventRecord(e->ev_chunk, e->s) != hipSuccess) return -5;
  e->chunk_pending = true;
  return 0;
}

// Waits for the last enqueued chunk (if wait, or if it has already finished) and retires the
// systems that are done: fills out[] (up to max_out), frees their rows and slots.
int engine_poll(Engine* e, bool wait, EngineDone* out, int max_out, int* n_out) {
  *n_out = 0;
  if (!e->chunk_pending) return 0;
  if (!wait) {
    const hipError_t q = hipEventQuery(e->ev_chunk);
    if (q == hipErrorNotReady) return 0;
    if (q != hipSuccess) return -5;
  } else if (hipEventSynchronize(e->ev_chunk) != hipSuccess) {
    return -5;
  }
  e->chunk_pending = false;
  if (e->probe_pending) {   // the sampled chunk's timed launches and bytes are complete
    probe_collect(e->d_probe, e->s);
    e->probe_pending = false;
  }
  int n = 0;
  for (int i = 0; i < e->max_sys && n < max_out; ++i) {
    if (!e->active[i] || status_of(*e, i).state != ST_DONE) continue;
    out[n].tag = e->tags[i];
    out[n].sum = status_of(*e, i);
    ++n;
    e->active[i] = 0;
    const SysDesc& d = e->h_sys[i];
    const int held = d.nunits * e->rv;
    for (int t = 0; t < held; ++t) e->tile_sys[d.tile_off + t] = -1;
    free_tiles_range(*e, d.tile_off, held);
    e->dirty = true;
  }
  *n_out = n;
  return 0;
}

void engine_usage(const Engine* e, int* active, int64_t* free_rows, int64_t* largest_free_rows) {
  int a = 0;
  for (int i = 0; i < e->max_sys; ++i) a += e->active[i] ? 1 : 0;
  int64_t f = 0, big = 0;
  for (const auto& kv : e->free_tiles) {
    f += kv.second;
    if (kv.second > big) big = kv.second;
  }
  *active = a;
  *free_rows = f * BS;
  *largest_free_rows = big * BS;
}

}  // namespace gsk
