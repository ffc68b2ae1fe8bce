// common.h -- wavefront and block helpers shared by the kernels (64-wide waves).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace eigupd {

// p[0 .. count) = 0 (a kernel, so that it can sit inside a captured graph)
__global__ void zero_ints_kernel(int* p, int count);

__device__ __forceinline__ bool update_cancelled(const DevState* st) {
  return __builtin_nontemporal_load(&st->status) != 0;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Inclusive prefix sum across the 64 lanes of a wave.
__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(v, off, 64);
    if (lane >= off) v += t;
  }
  return v;
}

__device__ __forceinline__ double wave_incl_max(double v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double t = __shfl_up(v, off, 64);
    if (lane >= off) v = fmax(v, t);
  }
  return v;
}

// Block-wide exclusive prefix sum for blocks of NT threads (NT/64 waves).
// sh needs NT/64 + 1 ints.  Returns the exclusive prefix; *total = block sum.
template <int NT>
__device__ __forceinline__ int block_excl_scan(int v, int* sh, int* total) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int inc = wave_incl_scan(v);
  __syncthreads();
  if (lane == 63) sh[wv] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int i = 0; i < NW; ++i) {
      const int t = sh[i];
      sh[i] = s;
      s += t;
    }
    sh[NW] = s;
  }
  __syncthreads();
  const int res = sh[wv] + inc - v;
  *total = sh[NW];
  return res;
}

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < NW; ++i) s += sh[i];
  return s;
}

template <int NT>
__device__ __forceinline__ double block_max(double v, double* sh) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double s = sh[0];
  for (int i = 1; i < NW; ++i) s = fmax(s, sh[i]);
  return s;
}

// 1/y to within about one ulp: hardware reciprocal estimate refined by two
// Newton-Raphson steps r <- r + r (1 - y r).  Returns 0 for y == 0.
__device__ __forceinline__ double recip(double y) {
  double r = __builtin_amdgcn_rcp(y);
  double e = fma(-y, r, 1.0);
  r = fma(r, e, r);
  e = fma(-y, r, 1.0);
  r = fma(r, e, r);
  return (y != 0.0) ? r : 0.0;
}

}  // namespace eigupd
