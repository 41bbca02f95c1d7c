// GS(p) row scaling, CSR validation and the standalone sparse product y = A x.
//
// GS(p) (section 1; section 2, eq. (2)) is gs_csr_tile (gsk_dev.hpp) over one tile of rows per
// workgroup. HBM traffic per row: read val (8/entry) and row_ptr (4), read b (8), write val
// (8/entry), b (8), and the optional norm/weight (8 each).
#include "gsk_host.hpp"

namespace gsk {

__global__ __launch_bounds__(64) void k_clear_flags(int* flags) {
  if (threadIdx.x < 16) flags[threadIdx.x] = 0;
}

__global__ __launch_bounds__(BS) void k_validate(const int* __restrict__ rp,
                                                 const int* __restrict__ ci, int n, int64_t nnz,
                                                 int* flags) {
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
    const int c = ci[k];
    if (c < 0 || c >= n) bad = true;
  }
  if (bad) atomicOr(&flags[0], 1);
}

hipError_t launch_clear_flags(int* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(64), 0, s, flags);
  return hipGetLastError();
}

hipError_t launch_validate(const Csr& A, int* flags, hipStream_t s) {
  int64_t work = A.nnz > (int64_t)A.n + 1 ? A.nnz : (int64_t)A.n + 1;
  int64_t blocks = (work + BS - 1) / BS;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_validate, dim3((unsigned)blocks), dim3(BS), 0, s, A.rp, A.ci, A.n, A.nnz,
                     flags);
  return hipGetLastError();
}

__global__ __launch_bounds__(BS) void k_gs_scale(const int* __restrict__ rp,
                                                 const int* __restrict__ ci,
                                                 const double* __restrict__ val,
                                                 const double* __restrict__ b, int n, int p,
                                                 int tiles, double* val_out, double* b_out,
                                                 double* __restrict__ norm_out,
                                                 double* __restrict__ weight_out, int* flags) {
  (void)ci;
  if (flags[0]) return;  // invalid CSR: touch nothing
  const int tile = logical_block();
  if (tile >= tiles) return;
  __shared__ GsLds L;
  const int row0 = tile * BS;
  bool zero = false, nonfinite = false;
  gs_csr_tile(rp, val, b, p, row0, min(BS, n - row0), val_out, b_out, norm_out, weight_out, L,
              zero, nonfinite);
  if (zero) atomicOr(&flags[1], 1);
  if (nonfinite) atomicOr(&flags[2], 1);
}

hipError_t launch_gs_scale(const Csr& A, const double* b, int p, double* val_out, double* b_out,
                           double* norm, double* weight, int* flags, hipStream_t s) {
  const int tiles = (A.n + BS - 1) / BS;
  const int grid = (tiles + 7) / 8 * 8;
  hipLaunchKernelGGL(k_gs_scale, dim3(grid), dim3(BS), 0, s, A.rp, A.ci, A.val, b, A.n, p, tiles,
                     val_out, b_out, norm, weight, flags);
  return hipGetLastError();
}

template <class Op>
__global__ __launch_bounds__(BS) void k_spmv(Op op, const double* __restrict__ x,
                                             double* __restrict__ y, int n, int tiles) {
  const int tile = logical_block();
  if (tile >= tiles) return;
  __shared__ typename Op::Lds L;
  const int row0 = tile * BS;
  const int nrows = min(BS, n - row0);
  const double v = op.tile(row0, nrows, GatherX{x}, L);
  if ((int)threadIdx.x < nrows) y[row0 + threadIdx.x] = v;
}

hipError_t launch_spmv(const Mat& A, const double* x, double* y, hipStream_t s) {
  const int tiles = (A.n + BS - 1) / BS;
  const int grid = (tiles + 7) / 8 * 8;
  if (A.kind == MAT_STENCIL)
    hipLaunchKernelGGL(k_spmv<StencilOp>, dim3(grid), dim3(BS), 0, s, A.stencil_op(), x, y, A.n,
                       tiles);
  else
    hipLaunchKernelGGL(k_spmv<CsrOp>, dim3(grid), dim3(BS), 0, s, A.csr_op(), x, y, A.n, tiles);
  return hipGetLastError();
}

// One row per thread: place each stored entry of row i in the plane of its offset from i
// (-nx*ny, -nx, -1, 0, +1, +nx, +nx*ny, each only where that neighbour is inside the grid),
// zero the planes the row does not use. Any other column, or a repeated position, is an error.
__global__ __launch_bounds__(BS) void k_stencil_from_csr(const int* __restrict__ rp,
                                                         const int* __restrict__ ci,
                                                         const double* __restrict__ val, int n,
                                                         int nx, int ny, int nz,
                                                         double* __restrict__ coef, int* flags) {
  if (flags[0]) return;
  const int64_t gi = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (gi >= n) return;
  const int i = (int)gi;
  const int ix = i % nx;
  const int rest = i / nx;
  const int iy = rest % ny;
  const int iz = rest / ny;
  const int nxy = nx * ny;
  const bool three = nz > 1;
  double v[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // -z, -y, -x, centre, +x, +y, +z
  unsigned seen = 0;
  bool bad = false;
  for (int k = rp[i]; k < rp[i + 1]; ++k) {
    const int d = ci[k] - i;
    int pl = -1;
    if (three && d == -nxy && iz > 0) pl = 0;
    else if (d == -nx && iy > 0) pl = 1;
    else if (d == -1 && ix > 0) pl = 2;
    else if (d == 0) pl = 3;
    else if (d == 1 && ix < nx - 1) pl = 4;
    else if (d == nx && iy < ny - 1) pl = 5;
    else if (three && d == nxy && iz < nz - 1) pl = 6;
    if (pl < 0 || (seen & (1u << pl))) {
      bad = true;
      continue;
    }
    seen |= 1u << pl;
    v[pl] = val[k];
  }
  if (bad) atomicOr(&flags[3], 1);
  if (three) {
#pragma unroll
    for (int q = 0; q < 7; ++q) coef[(size_t)q * n + i] = v[q];
  } else {
#pragma unroll
    for (int q = 0; q < 5; ++q) coef[(size_t)q * n + i] = v[q + 1];
  }
}

hipError_t launch_stencil_from_csr(const Csr& A, int nx, int ny, int nz, double* coef,
                                   int* flags, hipStream_t s) {
  const int grid = (A.n + BS - 1) / BS;
  hipLaunchKernelGGL(k_stencil_from_csr, dim3(grid), dim3(BS), 0, s, A.rp, A.ci, A.val, A.n, nx,
                     ny, nz, coef, flags);
  return hipGetLastError();
}

}  // namespace gsk
