// Deterministic block reductions shared by the vector kernels of the solo
// solvers and the cross-request batched ones: a fixed chunk per block, a fixed
// summation order, so every dot product is bitwise reproducible.
#pragma once

#include "dgs_internal.h"

namespace dgs {
namespace {

constexpr int kDotThreads = 256;

__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
  }
  __syncthreads();
  return t;  // valid on thread 0
}

// Two-stage dot products: the vector is cut into multidot_blocks(n) fixed
// chunks; block b writes partial[b * m + i] = (its chunk of V_i) . w, eight
// vectors per pass, and one block per i then sums the partials in a fixed
// order.  The fused variants first apply w -= sum_i coef_i V_i on the same
// chunk (each thread updates the points it later reads back itself, so no
// barrier is needed between the two phases).
constexpr int kDotGroup = 8;

template <int G>
__device__ __forceinline__ void group_store(double (&v)[G], double* red, double* out, int count) {
  constexpr int W = kDotThreads / 64;
#pragma unroll
  for (int q = 0; q < G; ++q)
    for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_down(v[q], off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < G; ++q) red[q * W + wave] = v[q];
  }
  __syncthreads();
  if ((int)threadIdx.x < count) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) t += red[threadIdx.x * W + w];
    out[threadIdx.x] = t;
  }
  __syncthreads();
}

__device__ __forceinline__ void chunk_dots(const double* __restrict__ V, long long ldv, int m,
                                           const double* w, long long start, long long end,
                                           double* red, double* __restrict__ partial) {
  for (int i0 = 0; i0 < m; i0 += kDotGroup) {
    double acc[kDotGroup];
#pragma unroll
    for (int q = 0; q < kDotGroup; ++q) acc[q] = 0.0;
    for (long long g = start + threadIdx.x; g < end; g += kDotThreads) {
      const double wg = w[g];
#pragma unroll
      for (int q = 0; q < kDotGroup; ++q)
        if (i0 + q < m) acc[q] += V[(long long)(i0 + q) * ldv + g] * wg;
    }
    group_store<kDotGroup>(acc, red, partial + (long long)blockIdx.x * m + i0,
                           m - i0 < kDotGroup ? m - i0 : kDotGroup);
  }
}

}  // namespace
}  // namespace dgs
