// Device-side building blocks shared by the gsk kernels (gfx950, wave64).
//
//  * Launch geometry: every Krylov kernel runs one workgroup of BS threads per contiguous
//    block of rows. The number of workgroups is a multiple of 8 and workgroup ids are
//    remapped so that the 8 XCDs (which receive workgroups round-robin) each own one
//    contiguous eighth of the rows; the neighbours a stencil row gathers then sit in the
//    same XCD's L2.
//  * Deterministic reductions without cross-workgroup synchronisation: per-thread partial
//    sums -> wave butterfly -> LDS across the waves -> one partial per workgroup, stored with
//    plain stores. A separate small "finalize" launch (one workgroup per reduced value) sums
//    the partials in a fixed order after the kernel boundary has made them visible, and
//    updates the solver's device-resident scalars. No fences, no atomics, no floating-point
//    atomics: repeated runs are bitwise identical.
//  * CSR tile product: a tile of BS rows stages val*x products in LDS with coalesced loads,
//    then each thread sums its own row sequentially in storage order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gsk {

constexpr int BS = 256;             // threads per workgroup (4 waves)
constexpr int WAVES = BS / 64;
constexpr int TILE_NNZ = BS * 8;    // LDS product slots per tile (8 per row on average)
constexpr int MMAX = 64;            // largest GMRES restart length
constexpr int NC_MAX = MMAX + 2;    // most values reduced in one launch
// Partials one thread of a finalize launch loads at once per column: SUM_BATCH, or in the single
// solvers' finalize launches for sums of more than SUM_BATCH * BS partials (a large system has
// tens of thousands of tiles) sum_batch<NC>() for NC columns (at most 128 values in flight per
// thread; those launches are instantiated for both, so that a small sum keeps the short
// kernel). A thread adds its partials t, t + BS, t + 2 BS, ... in that order whatever
// the batch, so the batch changes the number of memory round trips of a sum, not its value.
constexpr int SUM_BATCH = 8;
template <int NC>
constexpr int sum_batch() {
  return NC <= 4 ? 32 : 16;
}

// acc[c] += partials[c * stride + l] for l = t, t + BS, ... < count, in that order, loading SB
// values per column before adding them.
// The thread's index t in [0, BS) is an argument, so that the split finalize (split_sums) can
// run the thread of index t of the one-workgroup sum in another workgroup.
template <int NC, int SB>
__device__ inline void sweep_partials_of(const double* __restrict__ partials, int count,
                                         int stride, int t, double (&acc)[NC]) {
  for (int base = 0; base < count; base += SB * BS) {
    double v[NC][SB];
#pragma unroll
    for (int q = 0; q < SB; ++q) {
      const int l = base + q * BS + t;
#pragma unroll
      for (int c = 0; c < NC; ++c) v[c][q] = l < count ? partials[(size_t)c * stride + l] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int q = 0; q < SB; ++q) acc[c] += v[c][q];
  }
}

template <int NC, int SB>
__device__ inline void sweep_partials(const double* __restrict__ partials, int count, int stride,
                                      double (&acc)[NC]) {
  sweep_partials_of<NC, SB>(partials, count, stride, (int)threadIdx.x, acc);
}

// Solver state machine (Ctl::state)
enum : int {
  ST_INIT = 0,        // initial residual pending
  ST_RUNNING = 1,     // iterating
  ST_CYCLE_END = 2,   // GMRES: cycle finished, x update + true residual pending
  ST_HALF = 3,        // Bi-CGSTAB: half-step exit, x += alpha p pending
  ST_VERIFY = 4,      // true-residual check pending
  ST_FINAL = 5,       // breakdown: final true residual pending, status already set
  ST_DONE = 6,        // finished; status valid
  ST_SCALE = 7,       // batch engine: GS(p) of the system pending
  ST_ROLLBACK = 8,    // mixed Bi-CGSTAB engine: x back to its value at the last run's start
  ST_FP64START = 9,   // mixed Bi-CGSTAB engine: FP64 continuation, true residual pending
};

enum : int { S_CONVERGED = 0, S_MAXIT = 1, S_BREAKDOWN = 2, S_STAGNATED = 3 };

// Which breakdown test fired (Summary::brk)
enum : int { BRK_NONE = 0, BRK_SIGMA = 1, BRK_OMEGA = 2, BRK_RHO = 3, BRK_GIVENS = 4 };

// Kernel classes for the measurement hook (same numbering as GSK_KCLASS_* in gsk.h).
enum : int {
  KC_NONE = 0, KC_GMRES_A = 1, KC_GMRES_B = 2, KC_GMRES_C = 3, KC_BICG_P = 4, KC_BICG_S = 5,
  KC_BICG_U = 6, KC_RESIDUAL = 7, KC_GMRES_X = 8, KC_BATCH_P = 9, KC_BATCH_S = 10,
  KC_BATCH_U = 11, KC_COUNT = 12
};

// Measurement slots: a launch that the host chose to time carries a slot number; if it does
// work (rather than returning at once because the solve has moved on), thread 0 of workgroup 0
// stores its algorithmic bytes there. Zeroed by the init kernel.
constexpr int PROBE_SLOTS = 2048;
struct ProbeSlots {
  double bytes[PROBE_SLOTS];
};

// Host-visible summary copied back after each cycle / chunk.
struct Summary {
  int state, status, iters, restarts, half, fails, steps, brk;
  int fp64_from;   // mixed Bi-CGSTAB: iterations before the FP64 continuation (0: none)
  int pad0;
  double relres_rec, relres_true;
};

// Control block living at the start of the workspace. Written only by the kernels
// (its first fields are set by an init kernel, never by a memset).
struct Ctl {
  Summary sum;
  ProbeSlots probe;
  int maxit, m, j, k, claimed, first, has_w;
  int broke, happy;
  int bad;                   // batch engine: BAD_* bits of rejected system data
  int pad1;
  double tol, eps_b, ref, ratio;
  double last_rt;            // GMRES: relative true residual at the start of the cycle
  // Bi-CGSTAB scalars
  double rho, rho_old, alpha, omega, beta, rh_norm;
  // Split finalize of a large single-solver Bi-CGSTAB sum (split_sums): the wave sums of the
  // WAVES one-wave workgroups, WAVES consecutive entries per column, and the count of
  // workgroups that have stored theirs.
  double wsum[4 * WAVES];
  int fin_count;
  int pad2;
  // GMRES: lazy column scales, orthogonalisation coefficients, Hessenberg + Givens. The
  // pass-1 values of step j sit in slot j % 2: the single solver finalises step j-1 in the
  // launch that reduces the pass-1 sums of step j.
  double wnorm_pre[2];
  double sigma[MMAX + 1];
  double c1[2][MMAX + 1];
  double c2[MMAX + 1];
  double d1[MMAX + 1];     // c1_i sigma_i and c2_i sigma_i: the update weights of the stored
  double d2[MMAX + 1];     // (unnormalised) basis columns in the two CGS passes
  double H[(MMAX + 1) * MMAX];   // column-major, ld MMAX+1, rotated in place
  double Hraw[(MMAX + 1) * MMAX];// unrotated Hessenberg (for the Arnoldi entry point)
  double cs[MMAX], sn[MMAX], g[MMAX + 1], y[MMAX];
};

__device__ inline void mark_work(Ctl* c, int slot, double bytes) {
  if (slot >= 0 && blockIdx.x == 0 && threadIdx.x == 0) c->probe.bytes[slot] = bytes;
}

struct Geom {
  int nb;    // workgroups (multiple of 8)
  int rpb;   // rows per workgroup (multiple of BS)
};

// One tile of BS rows per workgroup, one row per thread; the workgroup count is rounded up to
// a multiple of 8 (the trailing workgroups own no rows).
inline Geom make_geom(int n) {
  const int tiles = (n + BS - 1) / BS;
  const int nb = (tiles + 7) / 8 * 8;
  return Geom{nb, BS};
}

// Workgroups of a launch whose workgroups own rpt consecutive tiles (rows_per_thread).
inline int grid_for(int n, int rpt) {
  const int tiles = (n + BS * rpt - 1) / (BS * rpt);
  return (tiles + 7) / 8 * 8;
}

// Logical workgroup index: XCD x (= blockIdx.x % 8) owns logical blocks
// [x*nb/8, (x+1)*nb/8), which are contiguous row ranges.
__device__ inline int logical_block() {
  const int nb = gridDim.x;
  const int b = blockIdx.x;
  return (b & 7) * (nb >> 3) + (b >> 3);
}

// Lane exchanges within one wave on the vector ALU (no LDS crossbar, unlike a shuffle through
// ds_bpermute). Within 16-lane rows they are DPP moves: quad_perm [1,0,3,2] and [2,3,0,1]
// give lane l ^ 1 and l ^ 2, row_ror:8 gives l ^ 8, and l ^ 4 takes row_ror:12 (lane l + 4)
// in lanes with bit 2 clear and row_ror:4 (lane l - 4) in the others. Across rows gfx950 has
// v_permlane16_swap / v_permlane32_swap: swap(a, b) exchanges the odd rows (upper half) of a
// with the even rows (lower half) of b.
template <int M>
__device__ inline int dpp_xor(int x, int lane) {
  static_assert(M == 1 || M == 2 || M == 4 || M == 8, "DPP exchange within a row");
  if constexpr (M == 1) return __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);
  if constexpr (M == 2) return __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);
  if constexpr (M == 8) return __builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false);
  if constexpr (M == 4) {
    const int up = __builtin_amdgcn_update_dpp(0, x, 0x12C, 0xF, 0xF, false);   // lane l + 4
    const int dn = __builtin_amdgcn_update_dpp(0, x, 0x124, 0xF, 0xF, false);   // lane l - 4
    return (lane & 4) ? dn : up;
  }
  return x;
}

// (a', b') = swap(a, b) on both 32-bit halves of a double: a' keeps a in the lower half of
// the lane group (row pair for M = 16, wave half for M = 32) and takes b's lower half in the
// upper one; b' takes a's upper half in the lower one and keeps b in the upper one.
template <int M>
__device__ inline void lane_swap(double& a, double& b) {
  static_assert(M == 16 || M == 32, "swap across rows");
  const unsigned alo = __double2loint(a), ahi = __double2hiint(a);
  const unsigned blo = __double2loint(b), bhi = __double2hiint(b);
  if constexpr (M == 32) {
    const auto lo = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
    a = __hiloint2double((int)hi[0], (int)lo[0]);
    b = __hiloint2double((int)hi[1], (int)lo[1]);
  } else {
    const auto lo = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
    a = __hiloint2double((int)hi[0], (int)lo[0]);
    b = __hiloint2double((int)hi[1], (int)lo[1]);
  }
}

// The value of x in lane (lane ^ M), M a power of two below 64.
template <int M>
__device__ inline double xor_lanes(double x, int lane) {
  if constexpr (M >= 16) {
    double a = x, b = x;
    lane_swap<M>(a, b);            // lower half: b = partner's x; upper half: a = partner's x
    return (lane & M) ? a : b;
  } else {
    const int lo = dpp_xor<M>(__double2loint(x), lane);
    const int hi = dpp_xor<M>(__double2hiint(x), lane);
    return __hiloint2double(hi, lo);
  }
}

template <int M>
struct WaveButterfly {
  __device__ static inline double run(double v, int lane) {
    v += xor_lanes<M>(v, lane);
    return WaveButterfly<M / 2>::run(v, lane);
  }
};
template <>
struct WaveButterfly<0> {
  __device__ static inline double run(double v, int) { return v; }
};

__device__ inline double wave_sum(double v) {
  return WaveButterfly<32>::run(v, threadIdx.x & 63);
}

// Reduce NC per-thread values over the workgroup and store them as this workgroup's partial
// (partials[c * nb + lb]). Only the first nc values are meaningful. lds must hold
// NC*WAVES doubles. All threads must call.
template <int NC>
__device__ inline void block_partials(double (&acc)[NC], int nc, double* __restrict__ partials,
                                      int nb, int lb, double* lds) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    if (c < nc) {
      double v = wave_sum(acc[c]);
      if (lane == 0) lds[c * WAVES + wave] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x < nc) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) s += lds[threadIdx.x * WAVES + w];
    partials[threadIdx.x * nb + lb] = s;
  }
}

// Reduce NV per-lane values (NV a power of two, <= 64) over the 64 lanes of a wave by
// recursive halving: at each step a lane keeps half of its values, sends the other half to
// its partner and adds what it receives, so the wave exchanges NV-1 + (6 - log2 NV) values
// instead of 6 NV. Afterwards lane l holds in v[0] the wave total of value number
// l >> (6 - log2 NV) (the remaining low lane bits are summed by a plain butterfly).
// Written as template recursion so that every array index is a compile-time constant and the
// values stay in registers.
template <int NV, int HALF, int BIT>
struct Halving {
  __device__ static inline void run(double (&v)[NV], int lane) {
    if constexpr (BIT >= 16) {
      // after the swap, a lane of the lower half holds its own v[k] and the partner's v[k],
      // a lane of the upper half the partner's v[k + HALF] and its own: add the two
#pragma unroll
      for (int k = 0; k < HALF; ++k) {
        double a = v[k], b = v[k + HALF];
        lane_swap<BIT>(a, b);
        v[k] = a + b;
      }
    } else {
      const bool hi = (lane & BIT) != 0;
#pragma unroll
      for (int k = 0; k < HALF; ++k) {
        const double send = hi ? v[k] : v[k + HALF];
        const double keep = hi ? v[k + HALF] : v[k];
        v[k] = keep + xor_lanes<BIT>(send, lane);
      }
    }
    Halving<NV, HALF / 2, BIT / 2>::run(v, lane);
  }
};

template <int NV, int BIT>
struct Halving<NV, 0, BIT> {
  __device__ static inline void run(double (&)[NV], int) {}
};

template <int NV>
__device__ inline double wave_halving_sum(double (&v)[NV]) {
  static_assert(NV >= 1 && NV <= 64 && (NV & (NV - 1)) == 0, "NV must be a power of two");
  const int lane = threadIdx.x & 63;
  Halving<NV, NV / 2, 32>::run(v, lane);
  return WaveButterfly<(NV > 1 ? 32 / NV : 32)>::run(v[0], lane);
}

template <int NV>
__device__ constexpr int halving_shift() {
  return NV >= 64 ? 0 : NV >= 32 ? 1 : NV >= 16 ? 2 : NV >= 8 ? 3 : NV >= 4 ? 4 : NV >= 2 ? 5 : 6;
}

// Workgroup version: partials[c * nb + lb] = workgroup total of value c, for c < nc <= NV.
// lds must hold NV*WAVES doubles. All threads must call.
template <int NV>
__device__ inline void block_halving_partials(double (&v)[NV], int nc,
                                              double* __restrict__ partials, int nb, int lb,
                                              double* lds) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  constexpr int SH = halving_shift<NV>();
  const double r = wave_halving_sum<NV>(v);
  if ((lane & ((1 << SH) - 1)) == 0) lds[(lane >> SH) * WAVES + wave] = r;
  __syncthreads();
  if ((int)threadIdx.x < nc) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) s += lds[threadIdx.x * WAVES + w];
    partials[threadIdx.x * nb + lb] = s;
  }
}

// Sum of partials[0..nb) in a fixed order (thread t adds t, t+BS, ... in turn; then the wave
// and workgroup trees). Every thread of the workgroup must call; all threads get the result.
template <int SB = SUM_BATCH>
__device__ inline double column_sum(const double* __restrict__ partials, int nb, double* lds) {
  // Each thread requests a batch of partials before it adds any of them, so a column of up to
  // a batch of BS-strided partials costs one memory round trip.
  double acc[1] = {0.0};
  sweep_partials<1, SB>(partials, nb, nb, acc);
  const double v = wave_sum(acc[0]);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < WAVES; ++w) s += lds[w];
  return s;
}

// In a single-workgroup finalize launch: out[c] = sum of partial column c (c < NC <= 8), all
// BS threads sweeping every column with independent loads; then the workgroup tree.
// out[c] = sum of the `count` partials of column c (column c starts at partials + c * stride),
// for c < NC <= 8, by one workgroup: every thread requests sum_batch values per column before
// it adds any, then the wave and workgroup trees. The result depends only on the column
// values and count, so a system's sums are the same wherever its partials sit.
template <int NC, int SB = SUM_BATCH>
__device__ inline void small_sums_strided(const double* __restrict__ partials, int count,
                                          int stride, double* out) {
  __shared__ double lds[8 * WAVES];
  double acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = 0.0;
  sweep_partials<NC, SB>(partials, count, stride, acc);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double v = wave_sum(acc[c]);
    if (lane == 0) lds[c * WAVES + wave] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < NC) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) s += lds[threadIdx.x * WAVES + w];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

template <int NC, int SB = SUM_BATCH>
__device__ inline void small_sums(const double* __restrict__ partials, int nb, double* out) {
  small_sums_strided<NC, SB>(partials, nb, nb, out);
}

// small_sums over WAVES workgroups of one wave, so that WAVES compute units read the partials:
// workgroup w runs the threads 64 w .. 64 w + 63 of the one-workgroup sum (the same additions
// in the same order, and the same wave tree) and stores its NC wave sums into c->wsum; the
// workgroup that stores last then adds the WAVES wave sums of each column in wave order, as
// the one-workgroup tree does. The result is small_sums' bit for bit. Returns true in that
// last workgroup, whose out[0..NC) then hold the sums (all its threads); false elsewhere.
// Launch with dim3(WAVES) x dim3(64); c->fin_count must be 0 at the launch (the last
// workgroup leaves it 0). No workgroup waits for another.
template <int NC, int SB>
__device__ inline bool split_sums(Ctl* c, const double* __restrict__ partials, int nb,
                                  double* out) {
  static_assert(NC <= 4, "c->wsum holds four columns");
  const int lane = threadIdx.x;
  const int w = blockIdx.x;
  double acc[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) acc[k] = 0.0;
  sweep_partials_of<NC, SB>(partials, nb, nb, w * 64 + lane, acc);
  double v[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) v[k] = wave_sum(acc[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NC; ++k)
      __hip_atomic_store(&c->wsum[k * WAVES + w], v[k], __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  }
  __threadfence();   // release: the wave sums reach device scope before the count
  int arrived = 0;
  if (lane == 0) arrived = atomicAdd(&c->fin_count, 1);
  arrived = __builtin_amdgcn_readfirstlane(arrived);
  if (arrived != WAVES - 1) return false;
  __threadfence();   // acquire: the other workgroups' wave sums
  if (lane < NC) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < WAVES; ++q)
      t += __hip_atomic_load(&c->wsum[lane * WAVES + q], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    out[lane] = t;
  }
  if (lane == 0) c->fin_count = 0;   // the next launch runs after this one has ended
  __syncthreads();
  return true;
}

// ---------------------------------------------------------------------------------------
// CSR tile product. Rows [row0, row0+nrows) with nrows <= BS; thread t gets row row0+t.
// gather(c) returns the (possibly recomputed) source-vector entry of column c.
// Products are rounded before they are added and each row is summed in storage order.
// Tiles whose nonzeros exceed the LDS slots fall back to a direct per-thread loop with
// the same rounding and order.
// ---------------------------------------------------------------------------------------
struct TileLds {
  int rp[BS + 1];
  double prod[TILE_NNZ];
};

template <class G, class V>
__device__ inline double csr_tile(const int* __restrict__ row_ptr, const int* __restrict__ col,
                                  const V* __restrict__ val, int row0, int nrows,
                                  const G& gather, TileLds& L) {
#pragma clang fp contract(off)
  const int t = threadIdx.x;
  for (int i = t; i <= nrows; i += BS) L.rp[i] = row_ptr[row0 + i];
  __syncthreads();
  const int p0 = L.rp[0];
  const int cnt = L.rp[nrows] - p0;
  double y = 0.0;
  if (cnt <= TILE_NNZ) {
    for (int k = t; k < cnt; k += BS) {
      const double a = (double)val[p0 + k];
      const double xv = gather(col[p0 + k]);
      L.prod[k] = a * xv;
    }
    __syncthreads();
    if (t < nrows) {
      const int e = L.rp[t + 1] - p0;
      for (int k = L.rp[t] - p0; k < e; ++k) y += L.prod[k];
    }
  } else {
    if (t < nrows) {
      const int e = L.rp[t + 1];
      for (int k = L.rp[t]; k < e; ++k) {
        const double prod = (double)val[k] * gather(col[k]);
        y += prod;
      }
    }
  }
  __syncthreads();   // LDS is reused by the next tile
  return y;
}

// ---------------------------------------------------------------------------------------
// GS(p) row scaling (section 1; section 2, eq. (2)): row i of A and b_i are divided by
// ||a_i||_p = (sum_j |a_ij|^p)^(1/p). Each row is summed in storage order, the same order and
// rounding as a sequential loop (p = 1 adds |a|, p = 2 adds a*a rounded); the stop-test weight
// of the row is ||a_i||_p / ||a_i||_2.
// ---------------------------------------------------------------------------------------
__device__ inline double abs_pow(double a, int p) {
  if (p == 1) return fabs(a);
  if (p == 2) return a * a;
  return pow(fabs(a), (double)p);
}

__device__ inline double root_p(double s, int p) {
  if (p == 1) return s;
  if (p == 2) return sqrt(s);
  return pow(s, 1.0 / (double)p);
}

struct GsLds {
  int rp[BS + 1];
  double val[TILE_NNZ];
  int row[TILE_NNZ];
  double scale[BS];
};

// One tile of a CSR matrix (rows row0 .. row0+nrows-1, thread t owns row row0+t): the tile's
// values are staged in LDS with coalesced loads, each thread sums its row, and the scaled
// values are written back coalesced (and, if val32 is given, also rounded to FP32). A row that
// is zero or non-finite sets the flag and leaves its outputs unwritten. All threads of the
// workgroup must call.
__device__ inline void gs_csr_tile(const int* __restrict__ rp, const double* __restrict__ val,
                                   const double* __restrict__ b, int p, int row0, int nrows,
                                   double* val_out, double* b_out, double* __restrict__ norm_out,
                                   double* __restrict__ weight_out, GsLds& L, bool& zero,
                                   bool& nonfinite, float* __restrict__ val32 = nullptr) {
#pragma clang fp contract(off)
  const int t = threadIdx.x;
  for (int i = t; i <= nrows; i += BS) L.rp[i] = rp[row0 + i];
  __syncthreads();
  const int p0 = L.rp[0];
  const int cnt = L.rp[nrows] - p0;
  const bool staged = cnt <= TILE_NNZ;
  if (staged) {
    for (int k = t; k < cnt; k += BS) L.val[k] = val[p0 + k];
    __syncthreads();
  }
  double nrm = 0.0;
  if (t < nrows) {
    const int ks = L.rp[t] - p0, ke = L.rp[t + 1] - p0;
    double sp = 0.0, s2 = 0.0;
    for (int k = ks; k < ke; ++k) {
      const double a = staged ? L.val[k] : val[p0 + k];
      if (!isfinite(a)) nonfinite = true;
      sp += abs_pow(a, p);
      s2 += a * a;
      if (staged) L.row[k] = t;
    }
    const double bi = b[row0 + t];
    if (!isfinite(bi)) nonfinite = true;
    if (sp == 0.0) zero = true;
    if (!nonfinite && !zero) {
      nrm = root_p(sp, p);
      if (!isfinite(nrm) || !isfinite(s2)) nonfinite = true;
    }
    const bool ok = !nonfinite && !zero;
    if (ok) {
      b_out[row0 + t] = bi / nrm;
      if (norm_out) norm_out[row0 + t] = nrm;
      if (weight_out) weight_out[row0 + t] = nrm / sqrt(s2);
      if (!staged)
        for (int k = ks; k < ke; ++k) {
          const double a = val[p0 + k] / nrm;
          val_out[p0 + k] = a;
          if (val32) val32[p0 + k] = (float)a;
        }
    }
    L.scale[t] = ok ? nrm : 0.0;
  }
  if (staged) {
    __syncthreads();
    for (int k = t; k < cnt; k += BS) {
      const double d = L.scale[L.row[k]];
      if (d != 0.0) {
        const double a = L.val[k] / d;
        val_out[p0 + k] = a;
        if (val32) val32[p0 + k] = (float)a;
      }
    }
  }
  __syncthreads();   // LDS is reused by the caller's next tile
}

// One row i of a 5/7-point stencil matrix held as coefficient planes (stride ldp): the present
// positions are summed in the CSR column order, so the norm, weight and scaled values equal
// those of the CSR form bit for bit (an absent position's coefficient, 0, is scaled to 0).
// If c32 is given, the scaled coefficients are also stored rounded to FP32 (planes of stride
// ldp32).
__device__ inline void gs_stencil_row(const double* __restrict__ coef, size_t ldp, int n,
                                      int nx, int ny, int nz, const double* __restrict__ b,
                                      int p, int i, double* coef_out, double* b_out,
                                      double* __restrict__ weight_out, bool& zero,
                                      bool& nonfinite, float* __restrict__ c32 = nullptr,
                                      size_t ldp32 = 0) {
#pragma clang fp contract(off)
  const int ix = i % nx;
  const int rest = i / nx;
  const int iy = rest % ny;
  const int iz = rest / ny;
  const bool three = nz > 1;
  const bool in[7] = {three && iz > 0, iy > 0,      ix > 0, true,
                      ix < nx - 1,     iy < ny - 1, three && iz < nz - 1};
  const int planes = three ? 7 : 5;
  double c[7];
  double sp = 0.0, s2 = 0.0;
  bool bad = false;
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    const int plane = three ? q : q - 1;
    c[q] = (plane >= 0 && plane < planes) ? coef[(size_t)plane * ldp + i] : 0.0;
    if (plane >= 0 && plane < planes && !isfinite(c[q])) bad = true;
    if (in[q]) {
      sp += abs_pow(c[q], p);
      s2 += c[q] * c[q];
    }
  }
  const double bi = b[i];
  if (!isfinite(bi)) bad = true;
  bool z = sp == 0.0;
  double nrm = 0.0;
  if (!bad && !z) {
    nrm = root_p(sp, p);
    if (!isfinite(nrm) || !isfinite(s2)) bad = true;
  }
  if (bad) nonfinite = true;
  if (z) zero = true;
  if (bad || z) return;
  b_out[i] = bi / nrm;
  if (weight_out) weight_out[i] = nrm / sqrt(s2);
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    const int plane = three ? q : q - 1;
    if (plane >= 0 && plane < planes) {
      const double a = c[q] / nrm;
      coef_out[(size_t)plane * ldp + i] = a;
      if (c32) c32[(size_t)plane * ldp32 + i] = (float)a;
    }
  }
}

// A gather supplies the source-vector entry of a column in two steps: load(col) fetches the
// raw operands (Raw), value(raw) combines them; g(col) == value(load(col)). Splitting the two
// lets a kernel issue every load before it combines anything. T is the storage type of the
// vector (double, or float for the FP32 inner solves); arithmetic is in double.
template <class T>
struct GatherXT {
  const T* __restrict__ x;
  typedef T Raw;
  __device__ Raw load(int c) const { return x[c]; }
  __device__ double value(Raw v) const { return (double)v; }
  __device__ double operator()(int c) const { return (double)x[c]; }
};
using GatherX = GatherXT<double>;

// ---------------------------------------------------------------------------------------
// Matrix operators. Every kernel that multiplies by A is templated on one of these:
//   typename Lds                                per-workgroup shared scratch
//   double tile(row0, nrows, gather, lds)       (A g)_row for row = row0 + threadIdx.x, valid
//                                               when threadIdx.x < nrows; all threads call it
//   double bytes                                 algorithmic bytes of one read of A
// ---------------------------------------------------------------------------------------
//
// Besides tile(), an operator offers the product in two phases, load() and finish(), so a
// kernel can put other loads between the two (see k_gmres_a); finish(load(...)) == tile().
// nrows >= 1 in every call. V is the storage type of the matrix values (double, or float for
// the FP32 copy the mixed-precision GMRES multiplies by); products and sums are in double.
template <class V>
struct CsrOpT {
  const int* rp;
  const int* ci;
  const V* val;
  typedef TileLds Lds;
  static constexpr bool kRowwise = false;   // tiles share LDS: one tile at a time
  template <class G>
  struct Pre {};   // a CSR tile stages its nonzeros through LDS behind barriers: nothing ahead
  template <class G>
  __device__ double tile(int row0, int nrows, const G& g, Lds& L) const {
    return csr_tile(rp, ci, val, row0, nrows, g, L);
  }
  template <class G>
  __device__ Pre<G> load(int, int, const G&) const { return Pre<G>{}; }
  template <class G>
  __device__ double finish(const Pre<G>&, int row0, int nrows, const G& g, Lds& L) const {
    return tile(row0, nrows, g, L);
  }
};

using CsrOp = CsrOpT<double>;

struct EmptyLds {
  int unused;
};

// Structured 5-point (nz == 1) or 7-point stencil on an nx x ny x nz grid, x fastest.
// coef holds one plane of n values per stencil position, in the CSR column order
// -z, -y, -x, centre, +x, +y, +z (-z and +z absent in 2D); neighbours outside the grid are
// skipped. Each row is summed in that order with every product rounded before it is added,
// so the result equals the CSR product of the same matrix bit for bit.
template <class V, bool NT = false>
struct StencilOpT {
  const V* coef;
  int n, nx, ny, nz;
  size_t ldp;    // stride between coefficient planes (n for a caller's matrix)
  typedef EmptyLds Lds;
  static constexpr bool kRowwise = true;    // rows are independent: several tiles at once
  // Position q of a row: -z, -y, -x, centre, +x, +y, +z. load() fetches every coefficient and
  // neighbour without a branch, so that all loads are in flight together: the neighbour index
  // is i + offset clamped to [0, n), a valid address whatever the position, and a position
  // outside the grid (or -z/+z in 2D) is flagged absent and its values are never used.
  template <class G>
  struct Pre {
    V c[7];
    typename G::Raw x[7];
    unsigned present;
    // The gathered operands of the centre position: a row's own entries (rows of the tile).
    __device__ const typename G::Raw& centre() const { return x[3]; }
  };
  template <class G>
  __device__ Pre<G> load(int row0, int nrows, const G& g) const {
    Pre<G> p;
    const int t = threadIdx.x;
    // rows past the tile repeat its last row; a tile past the end of the matrix reads row n-1
    const int i = min(row0 + max(0, min(t, nrows - 1)), n - 1);
    const int ix = i % nx;
    const int rest = i / nx;
    const int iy = rest % ny;
    const int iz = rest / ny;
    const int nxy = nx * ny;
    const bool three = nz > 1;
    const bool in[7] = {three && iz > 0, iy > 0,      ix > 0, true,
                        ix < nx - 1,     iy < ny - 1, three && iz < nz - 1};
    const int off[7] = {-nxy, -nx, -1, 0, 1, nx, nxy};
    p.present = 0;
#pragma unroll
    for (int q = 0; q < 7; ++q) {
      const int plane = three ? q : (q == 0 ? 0 : q == 6 ? 4 : q - 1);
      if constexpr (NT) p.c[q] = __builtin_nontemporal_load(coef + (size_t)plane * ldp + i);
      else p.c[q] = coef[(size_t)plane * ldp + i];
      const long long k = (long long)i + off[q];
      p.x[q] = g.load((int)(k < 0 ? 0 : k >= n ? n - 1 : k));
      p.present |= in[q] ? 1u << q : 0u;
    }
    return p;
  }
  // Sum in position order with every product rounded; an absent position adds +0.0, which
  // leaves the sum unchanged (a sum that starts at +0.0 never becomes -0.0), so the result
  // equals the CSR product of the same matrix bit for bit.
  template <class G>
  __device__ double finish(const Pre<G>& p, int, int nrows, const G& g, Lds&) const {
#pragma clang fp contract(off)
    if ((int)threadIdx.x >= nrows) return 0.0;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 7; ++q)
      s += (p.present >> q) & 1u ? (double)p.c[q] * g.value(p.x[q]) : 0.0;
    return s;
  }
  template <class G>
  __device__ double tile(int row0, int nrows, const G& g, Lds& L) const {
    return finish(load(row0, nrows, g), row0, nrows, g, L);
  }
};

using StencilOp = StencilOpT<double>;

// The same product with the gathered vector's x and y neighbours read from an LDS window: the
// tile's rows and one x-line on either side (clipped to the matrix) are loaded once and
// formed into LDS; a row takes -y, -x, centre, +x and +y from there and gathers only -z and +z
// from global memory. One tile per workgroup (one row per thread), x-lines of at most kWinNx
// points; finish() holds a workgroup barrier, so every thread of the workgroup calls it. Each
// row is summed in position order with the roundings of StencilOpT: the same bits.
constexpr int kWinNx = 256;

template <class V, bool NT = false>
struct StencilWinOpT {
  const V* coef;
  int n, nx, ny, nz;
  size_t ldp;
  struct Lds {
    double g[BS + 2 * kWinNx];
  };
  static constexpr bool kRowwise = true;
  static constexpr int kWin = (BS + 2 * kWinNx) / BS;   // window loads per thread
  template <class G>
  struct Pre {
    V c[7];
    typename G::Raw z[2];
    typename G::Raw w[kWin];
    unsigned present;
    int i, w0, wn;
  };
  template <class G>
  __device__ Pre<G> load(int row0, int nrows, const G& g) const {
    Pre<G> p;
    const int t = threadIdx.x;
    const int i = min(row0 + max(0, min(t, nrows - 1)), n - 1);
    const int ix = i % nx;
    const int rest = i / nx;
    const int iy = rest % ny;
    const int iz = rest / ny;
    const int nxy = nx * ny;
    const bool three = nz > 1;
    const bool in[7] = {three && iz > 0, iy > 0,      ix > 0, true,
                        ix < nx - 1,     iy < ny - 1, three && iz < nz - 1};
    p.present = 0;
#pragma unroll
    for (int q = 0; q < 7; ++q) {
      const int plane = three ? q : (q == 0 ? 0 : q == 6 ? 4 : q - 1);
      if constexpr (NT) p.c[q] = __builtin_nontemporal_load(coef + (size_t)plane * ldp + i);
      else p.c[q] = coef[(size_t)plane * ldp + i];
      p.present |= in[q] ? 1u << q : 0u;
    }
    p.z[0] = g.load(max(i - nxy, 0));
    p.z[1] = g.load(min(i + nxy, n - 1));
    const int r0 = min(row0, n - 1);
    p.w0 = max(0, r0 - nx);
    p.wn = min(n, r0 + BS + nx) - p.w0;
#pragma unroll
    for (int k = 0; k < kWin; ++k) p.w[k] = g.load(p.w0 + min(k * BS + t, p.wn - 1));
    p.i = i;
    return p;
  }
  template <class G>
  __device__ double finish(const Pre<G>& p, int, int nrows, const G& g, Lds& L) const {
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < kWin; ++k)
      if (k * BS + t < p.wn) L.g[k * BS + t] = g.value(p.w[k]);
    __syncthreads();
    if (t >= nrows) return 0.0;
    const int li = p.i - p.w0;
    double x[7];
    x[0] = g.value(p.z[0]);
    x[1] = L.g[max(li - nx, 0)];
    x[2] = L.g[max(li - 1, 0)];
    x[3] = L.g[li];
    x[4] = L.g[min(li + 1, p.wn - 1)];
    x[5] = L.g[min(li + nx, p.wn - 1)];
    x[6] = g.value(p.z[1]);
    double s = 0.0;
    {
#pragma clang fp contract(off)
#pragma unroll
      for (int q = 0; q < 7; ++q) s += (p.present >> q) & 1u ? (double)p.c[q] * x[q] : 0.0;
    }
    return s;
  }
};

// Reads columns of a column-major n x k basis stored as T (double or float) through one buffer
// descriptor: the column offset is a uniform scalar (i * ldv * sizeof(T) bytes) and the row
// offset a single per-lane 32-bit value, so a thread reading 30 columns of its row holds no
// per-column addresses. Requires the basis to span fewer than 2^31 bytes (checked on the
// host). Values are returned as double.
// NT: the loads carry the non-temporal cache policy (a basis much larger than the caches is
// streamed once per launch; keeping it out of the caches leaves room for the data that is
// reused). The values are the same either way.
template <class T, bool NT = false>
struct ColumnReaderT {
  __amdgpu_buffer_rsrc_t rsrc;
  int ld_bytes;
  static constexpr int kAux = NT ? 2 : 0;   // cache-policy operand: bit 1 = nt
  __device__ ColumnReaderT(const T* base, size_t ldv, int cols) {
    rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), (short)0,
                                             (int)(ldv * sizeof(T) * (size_t)cols), 0x00020000);
    ld_bytes = (int)(ldv * sizeof(T));
  }
  __device__ T raw(int col, int row) const {
    if constexpr (sizeof(T) == 8) {
      typedef unsigned int u2 __attribute__((ext_vector_type(2)));
      const u2 v = __builtin_amdgcn_raw_buffer_load_b64(rsrc, row * 8, col * ld_bytes, kAux);
      return __builtin_bit_cast(double, v);
    } else {
      const unsigned int v =
          __builtin_amdgcn_raw_buffer_load_b32(rsrc, row * 4, col * ld_bytes, kAux);
      return __builtin_bit_cast(float, v);
    }
  }
  __device__ double load(int col, int row) const { return (double)raw(col, row); }
};

// Same interface with plain 64-bit addressing, for bases of 2^31 bytes or more.
template <class T, bool NT = false>
struct PointerReaderT {
  const T* base;
  size_t ldv;
  __device__ PointerReaderT(const T* b, size_t l, int) : base(b), ldv(l) {}
  __device__ T raw(int col, int row) const {
    if constexpr (NT) return __builtin_nontemporal_load(base + (size_t)col * ldv + row);
    else return base[(size_t)col * ldv + row];
  }
  __device__ double load(int col, int row) const { return (double)raw(col, row); }
};

using ColumnReader = ColumnReaderT<double>;
using PointerReader = PointerReaderT<double>;

template <class T>
inline bool fits_buffer(size_t ldv, int cols) {
  return ldv * sizeof(T) * (size_t)cols < (size_t(1) << 31);
}

}  // namespace gsk
