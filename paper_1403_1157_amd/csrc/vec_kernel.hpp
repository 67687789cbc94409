// Vector kernels of the implicit (Newton-Krylov) time integrator: linear
// combinations and deterministic dot products over whole state vectors.
//
// Determinism: every dot product is summed in a fixed order that depends only on
// the vector length (each workgroup owns one contiguous range, its threads
// stride through it, a fixed butterfly combines the lanes of a wavefront and
// the wavefronts are added in order; the partials of the workgroups are added
// in order by a second kernel), so results are bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>

namespace cdg2 {

constexpr int VEC_NT = 256;    // threads per workgroup of the vector kernels
constexpr int DOT_NB = 512;    // workgroups of a dot-product pass
constexpr int DOT_W = 8;       // vectors per dot-product pass

// out = a0 x0 + a1 x1 + a2 x2 + a3 x3 (terms with a null vector are skipped);
// out may alias any input.
__global__ void __launch_bounds__(VEC_NT)
lincomb_kernel(size_t n, double* out, const double* x0, double a0, const double* x1, double a1,
               const double* x2, double a2, const double* x3, double a3) {
  for (size_t i = (size_t)blockIdx.x * VEC_NT + threadIdx.x; i < n; i += (size_t)gridDim.x * VEC_NT) {
    double v = x0 ? a0 * x0[i] : 0.0;
    if (x1) v += a1 * x1[i];
    if (x2) v += a2 * x2[i];
    if (x3) v += a3 * x3[i];
    out[i] = v;
  }
}

// Sum of one value over a workgroup of VEC_NT threads, result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* red) {
  static_assert(VEC_NT % 64 == 0, "whole wavefronts");
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < VEC_NT / 64; ++k) s += red[k];
  return s;
}

// Partial dot products of w with up to DOT_W vectors of the group blockIdx.y:
// vector j is V + j ld (j < k), or w itself for j == k when self != 0.
// part[j * DOT_NB + blockIdx.x].
__global__ void __launch_bounds__(VEC_NT)
dots_kernel(size_t n, const double* __restrict__ w, const double* __restrict__ V, size_t ld, int k, int self,
            double* __restrict__ part) {
  __shared__ double red[VEC_NT / 64];
  const int j0 = blockIdx.y * DOT_W;
  const int kk = k + (self ? 1 : 0);
  const size_t chunk = (n + DOT_NB - 1) / DOT_NB;
  const size_t lo = (size_t)blockIdx.x * chunk;
  const size_t hi = lo + chunk < n ? lo + chunk : n;
  double acc[DOT_W];
#pragma unroll
  for (int q = 0; q < DOT_W; ++q) acc[q] = 0.0;
  for (size_t i = lo + threadIdx.x; i < hi; i += VEC_NT) {
    const double wi = w[i];
#pragma unroll
    for (int q = 0; q < DOT_W; ++q) {
      const int j = j0 + q;
      if (j < k) acc[q] += wi * V[(size_t)j * ld + i];
      else if (j == k && self) acc[q] += wi * wi;
    }
  }
#pragma unroll
  for (int q = 0; q < DOT_W; ++q) {
    const int j = j0 + q;
    const double s = block_sum(acc[q], red);
    if (threadIdx.x == 0 && j < kk) part[(size_t)j * DOT_NB + blockIdx.x] = s;
  }
}

// out[j] = sum over the DOT_NB partials of dot j, in order; one workgroup per j.
__global__ void __launch_bounds__(VEC_NT) dots_reduce_kernel(const double* __restrict__ part, double* out) {
  __shared__ double red[VEC_NT / 64];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < DOT_NB; b += VEC_NT) s += part[(size_t)j * DOT_NB + b];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[j] = s;
}

// w -= scale * sum_{j<k} h[j] (V + j ld), h on the device.
__global__ void __launch_bounds__(VEC_NT)
multi_axpy_kernel(size_t n, double* w, const double* __restrict__ V, size_t ld, int k, const double* __restrict__ h,
                  double scale) {
  for (size_t i = (size_t)blockIdx.x * VEC_NT + threadIdx.x; i < n; i += (size_t)gridDim.x * VEC_NT) {
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += h[j] * V[(size_t)j * ld + i];
    w[i] -= scale * s;
  }
}

}  // namespace cdg2
