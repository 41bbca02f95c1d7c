// Measurement hook (not part of the method): the memory ceiling of a streaming kernel's mix of
// arrays on this device. k_stream_mix<R, W> reads R arrays and writes W arrays of n doubles
// with one row per thread in 256-row tiles (XCD-aware workgroup order, one 8-byte load per
// array and row) and reduces one value per tile through the wave and workgroup trees into a
// partial, as the solvers' streaming kernels do; it has no gathers and no control block. Its
// time for a mix such as the batch engine's P pass (7 coefficient planes and r, p, v, r^ read,
// p and v written) bounds what a kernel with that mix can reach.
#include "gsk_host.hpp"

namespace gsk {

template <int R, int W>
__global__ __launch_bounds__(BS) void k_stream_mix(double* __restrict__ buf, int64_t n,
                                                   double* __restrict__ partials) {
  __shared__ double red[WAVES];
  const int lb = logical_block();
  const int64_t i = (int64_t)lb * BS + threadIdx.x;
  const bool mine = i < n;
  double v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = mine ? buf[(size_t)r * n + i] : 0.0;
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) s += v[r];
  if (mine) {
#pragma unroll
    for (int w = 0; w < W; ++w) buf[(size_t)(R + w) * n + i] = s * (double)(w + 1);
  }
  const double t = wave_sum(s * v[0]);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) a += red[w];
    partials[lb] = a;
  }
}

template <int R, int W>
static hipError_t stream_mix(double* buf, int64_t n, int reps, float* best_ms, hipStream_t s) {
  const int64_t tiles = (n + BS - 1) / BS;
  const int grid = (int)((tiles + 7) / 8 * 8);
  double* partials = buf + (size_t)(R + W) * (size_t)n;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t err = hipEventCreate(&e0);
  if (err == hipSuccess) err = hipEventCreate(&e1);
  float best = -1.0f;
  for (int k = 0; err == hipSuccess && k <= reps; ++k) {   // launch 0 warms up
    hipExtLaunchKernelGGL(k_stream_mix<R, W>, dim3(grid), dim3(BS), 0, s, e0, e1, 0, buf, n,
                          partials);
    err = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (err == hipSuccess && k > 0 && (best < 0.0f || ms < best)) best = ms;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  *best_ms = best;
  return err;
}

// Supported mixes: (1, 0) a plain read, (1, 1) a copy, (6, 2) the Bi-CGSTAB U pass, (9, 1) the
// S pass, (11, 2) the P pass (7-point planes); -1 for any other.
int stream_mix_ms(int reads, int writes, int64_t n, double* buf, int reps, float* best_ms,
                  hipStream_t s) {
  hipError_t e;
  if (reads == 1 && writes == 0) e = stream_mix<1, 0>(buf, n, reps, best_ms, s);
  else if (reads == 1 && writes == 1) e = stream_mix<1, 1>(buf, n, reps, best_ms, s);
  else if (reads == 6 && writes == 2) e = stream_mix<6, 2>(buf, n, reps, best_ms, s);
  else if (reads == 9 && writes == 1) e = stream_mix<9, 1>(buf, n, reps, best_ms, s);
  else if (reads == 11 && writes == 2) e = stream_mix<11, 2>(buf, n, reps, best_ms, s);
  else return -1;
  return e == hipSuccess ? 0 : -5;
}

}  // namespace gsk
