// qtk.hip -- U = Q^T K (Sec. 2.1: U = Q^T K; Sec. 2.4 calls it L).
//
// Q is n-by-n column-major (leading dimension ldq >= n) and K n-by-k with
// k <= 8, so U is a skinny product bound by streaming Q from HBM once
// (8 n^2 bytes, 2 n^2 k flops).  A block of 256 threads owns CPB consecutive
// columns of Q (qtk_cpb: 2 to 8 with k): each thread takes the row pairs
// r = 2 tid + 1024 i and r + 512 (16-byte streaming loads, coalesced along the
// column, all issued before any is used; rows tid, tid + 256, ... when n or ldq
// is odd), combines them with K's rows, and the block reduces CPB*k partial
// sums at the end.  Measured at n = 8192, k = 2 this runs within 5% of the
// read-only streaming rate of the chip (eight columns per block and one row
// pair per step: 20% slower).
// Non-finite entries of U raise the sticky ST_NONFINITE bit.
#include "common.h"

namespace eigupd {

template <int K, int CPB>
__device__ __forceinline__ void qtk_body(const Work& w, int bid) {
  if (update_cancelled(w.st)) return;
  const int n = w.n;
  const int j0 = bid * CPB;
  double acc[CPB][K];
#pragma unroll
  for (int q = 0; q < CPB; ++q)
#pragma unroll
    for (int c = 0; c < K; ++c) acc[q][c] = 0.0;
  const double* __restrict__ Q = w.Q_in;
  const double* __restrict__ Km = w.K;
  const size_t ldq = (size_t)w.ldq;
  const int ncol = min(CPB, n - j0);
  if (!(n & 1) && !(ldq & 1) && !((uintptr_t)Q & 15)) {
    // rows r, r + 1 (r even) in one 16-byte load per column; two such pairs,
    // 512 rows apart, per step
    typedef double dv2 __attribute__((ext_vector_type(2)));
    for (int r0 = 2 * threadIdx.x; r0 < n; r0 += 1024) {
      dv2 v[2][CPB];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int q = 0; q < CPB; ++q) {
          const int r = r0 + 512 * h;
          v[h][q] = dv2{0.0, 0.0};
          if (q < ncol && r < n)
            v[h][q] = __builtin_nontemporal_load(
                reinterpret_cast<const dv2*>(Q + r + (size_t)(j0 + q) * ldq));
        }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = r0 + 512 * h;
        if (r >= n) break;
        double k0[K], k1[K];
#pragma unroll
        for (int c = 0; c < K; ++c) {
          k0[c] = Km[r + (size_t)c * w.ldk];
          k1[c] = Km[r + 1 + (size_t)c * w.ldk];
        }
#pragma unroll
        for (int q = 0; q < CPB; ++q)
#pragma unroll
          for (int c = 0; c < K; ++c)
            acc[q][c] = fma(v[h][q][1], k1[c], fma(v[h][q][0], k0[c], acc[q][c]));
      }
    }
  } else {
    for (int r = threadIdx.x; r < n; r += 256) {
      double kr[K];
#pragma unroll
      for (int c = 0; c < K; ++c) kr[c] = Km[r + (size_t)c * w.ldk];
#pragma unroll
      for (int q = 0; q < CPB; ++q) {
        const double v = (q < ncol) ? Q[r + (size_t)(j0 + q) * ldq] : 0.0;
#pragma unroll
        for (int c = 0; c < K; ++c) acc[q][c] = fma(v, kr[c], acc[q][c]);
      }
    }
  }
  __shared__ double red[4][CPB * K];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < CPB; ++q)
#pragma unroll
    for (int c = 0; c < K; ++c) {
      const double s = wave_sum(acc[q][c]);
      if (lane == 0) red[wv][q * K + c] = s;
    }
  __syncthreads();
  if (threadIdx.x < CPB * K) {
    const int e = threadIdx.x;
    const double s = red[0][e] + red[1][e] + red[2][e] + red[3][e];
    const int q = e / K, c = e % K;
    if (q < ncol) {
      w.U[(size_t)(j0 + q) * K + c] = s;
      if (!isfinite(s)) atomicOr(&w.st->status, ST_NONFINITE);
    }
  }
}

template <int K, int CPB>
__global__ __launch_bounds__(256) void qtk_kernel(Work w) {
  qtk_body<K, CPB>(w, blockIdx.x);
}

template <int K, int CPB>
__global__ __launch_bounds__(256) void qtk_group(Group g) {
  const int i = group_instance(g, blockIdx.x);
  qtk_body<K, CPB>(g.works[i], blockIdx.x - g.prefix[i]);
}

// Columns per block: each thread loads k entries of K per row pair and uses them
// for CPB columns, so CPB grows with k; measured at n = 8192 and 16384 (k = 1:
// 2; k = 2: 4; k >= 3: 8, within 2% of the best of {2, 4, 8} at both sizes).
constexpr int qtk_cpb(int k) { return (k == 1) ? 2 : (k == 2) ? 4 : 8; }

int qtk_blocks(int n, int k) { return (n + qtk_cpb(k) - 1) / qtk_cpb(k); }

template <int K>
static hipError_t qtk_launch(const Work& w, hipStream_t s) {
  constexpr int CPB = qtk_cpb(K);
  const int grid = (w.n + CPB - 1) / CPB;
  hipLaunchKernelGGL((qtk_kernel<K, CPB>), dim3(grid), dim3(256), 0, s, w);
  return hipGetLastError();
}

template <int K>
static hipError_t qtk_group_launch(const Group& g, int blocks, hipStream_t s) {
  hipLaunchKernelGGL((qtk_group<K, qtk_cpb(K)>), dim3(blocks), dim3(256), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_qtk(const Work& w, hipStream_t s) {
  switch (w.k) {
    case 1: return qtk_launch<1>(w, s);
    case 2: return qtk_launch<2>(w, s);
    case 3: return qtk_launch<3>(w, s);
    case 4: return qtk_launch<4>(w, s);
    case 5: return qtk_launch<5>(w, s);
    case 6: return qtk_launch<6>(w, s);
    case 7: return qtk_launch<7>(w, s);
    case 8: return qtk_launch<8>(w, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_qtk_group(int k, const Group& g, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  EIGUPD_SWITCH_K(k, qtk_group_launch, g, blocks, s)
}

}  // namespace eigupd
