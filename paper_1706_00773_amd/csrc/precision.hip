// precision.hip -- reduced-precision variants of the two dense products of an
// update, U = Q^T K (Sec. 2.1) and Q' = Q W (Sec. 2.4, eq. (10)), with FP64
// combination of the partial results.  The secular roots, the pole
// differences and the deflation tests stay in FP64.
//
// Operand splitting (from the FP64 operands):
//   FP32 mode   x = hi + lo + r, hi = fl32(x), lo = fl32(x - hi), |r| <~ 2^-48 |x|
//   BF16X3 mode x = b0 + b1 + b2 + r, b_{i+1} = bf16(x - b0 - ... - b_i),
//               |r| <~ 2^-24 |x|
// Products kept:
//   FP32        hi*hi (main) and hi*lo + lo*hi (cross terms, own accumulator)
//   BF16X3      every b_i*b_j with i + j <= 2 (six products, one accumulator;
//               the smaller products are issued first)
// The FP32 accumulators of a k-slice are added into FP64 accumulators after
// every slice, so FP32 rounding only ever acts on one slice's partial sums.
//
// U = Q^T K is a skinny product bound by streaming Q (k <= 8 columns), so its
// variant runs on the vector ALUs with the same splitting and FP32
// accumulation; the FP64 residual correction then restores it to FP64
// accuracy:  U = U_lo + lo(Q^T (K - Q U_lo)), with K - Q U_lo formed in FP64.
//
// Q' = Q W runs on the matrix cores, from operands split once per update
// into slice planes (split_w, split_qt):
//   FP32   v_mfma_f32_16x16x4_f32   (3 products per k-step)
//   BF16X3 v_mfma_f32_16x16x32_bf16 (6 products per k-step)
// Both use the output layout of the FP32-accumulating MFMAs on gfx950: lane l,
// register v holds row 4*(l/16) + v, column l%16 of the 16x16 tile.  A lane's
// operand fragment is a run of consecutive k (4 floats or 8 bf16) of one row
// of A and one column of B; the same k permutation is used for both, so the
// sum over k is unchanged.  LDS holds the split tiles k-contiguous: As[m][k],
// Bs[n][k], rows padded to 80 bytes so a 16-lane group's 16-byte fragment
// reads fall in distinct banks.
#include "common.h"

namespace eigupd {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------- splitting

__device__ __forceinline__ void split_f32(double x, float& hi, float& lo) {
  hi = (float)x;
  lo = (float)(x - (double)hi);
}

__device__ __forceinline__ unsigned short bf16_bits(float f) {
  const __bf16 h = (__bf16)f;
  return __builtin_bit_cast(unsigned short, h);
}

__device__ __forceinline__ float bf16_value(unsigned short b) {
  return __uint_as_float((unsigned)b << 16);
}

__device__ __forceinline__ void split_bf16x3(double x, unsigned short& b0, unsigned short& b1,
                                             unsigned short& b2) {
  b0 = bf16_bits((float)x);
  const double r1 = x - (double)bf16_value(b0);
  b1 = bf16_bits((float)r1);
  const double r2 = r1 - (double)bf16_value(b1);
  b2 = bf16_bits((float)r2);
}

// ---------------------------------------------------------- U = Q^T K (VALU)

// Output row j of U (column j of Q) for CPB consecutive columns per block.
// accumulate != 0 adds the result to U (the correction pass).
template <int K, int CPB, int P>
__global__ __launch_bounds__(256) void qtk_lp_kernel(Work w, const double* __restrict__ Km,
                                                     int ldk, int accumulate) {
  if (update_cancelled(w.st)) return;
  constexpr int CH = 8;  // rows per thread between FP64 promotions
  const int n = w.n;
  const int j0 = blockIdx.x * CPB;
  const int ncol = min(CPB, n - j0);
  const double* __restrict__ Q = w.Q_in;
  double acc[CPB][K];
  float lo32[CPB][K], cr32[CPB][K];
#pragma unroll
  for (int q = 0; q < CPB; ++q)
#pragma unroll
    for (int c = 0; c < K; ++c) {
      acc[q][c] = 0.0;
      lo32[q][c] = 0.0f;
      cr32[q][c] = 0.0f;
    }
  int cnt = 0;
  for (int r = threadIdx.x; r < n; r += 256) {
    if (P == EIG_GEMM_FP32_CORR) {
      float kh[K], kl[K];
#pragma unroll
      for (int c = 0; c < K; ++c) split_f32(Km[r + (size_t)c * ldk], kh[c], kl[c]);
#pragma unroll
      for (int q = 0; q < CPB; ++q) {
        float vh = 0.0f, vl = 0.0f;
        if (q < ncol) split_f32(Q[r + (size_t)(j0 + q) * n], vh, vl);
#pragma unroll
        for (int c = 0; c < K; ++c) {
          lo32[q][c] = fmaf(vh, kh[c], lo32[q][c]);
          cr32[q][c] = fmaf(vh, kl[c], fmaf(vl, kh[c], cr32[q][c]));
        }
      }
    } else {
      float k0[K], k1[K], k2[K];
#pragma unroll
      for (int c = 0; c < K; ++c) {
        unsigned short a, b, d;
        split_bf16x3(Km[r + (size_t)c * ldk], a, b, d);
        k0[c] = bf16_value(a);
        k1[c] = bf16_value(b);
        k2[c] = bf16_value(d);
      }
#pragma unroll
      for (int q = 0; q < CPB; ++q) {
        float v0 = 0.0f, v1 = 0.0f, v2 = 0.0f;
        if (q < ncol) {
          unsigned short a, b, d;
          split_bf16x3(Q[r + (size_t)(j0 + q) * n], a, b, d);
          v0 = bf16_value(a);
          v1 = bf16_value(b);
          v2 = bf16_value(d);
        }
#pragma unroll
        for (int c = 0; c < K; ++c) {
          float s = lo32[q][c];
          s = fmaf(v2, k0[c], s);
          s = fmaf(v1, k1[c], s);
          s = fmaf(v0, k2[c], s);
          s = fmaf(v1, k0[c], s);
          s = fmaf(v0, k1[c], s);
          s = fmaf(v0, k0[c], s);
          lo32[q][c] = s;
        }
      }
    }
    if (++cnt == CH) {
      cnt = 0;
#pragma unroll
      for (int q = 0; q < CPB; ++q)
#pragma unroll
        for (int c = 0; c < K; ++c) {
          acc[q][c] += (double)lo32[q][c] + (double)cr32[q][c];
          lo32[q][c] = 0.0f;
          cr32[q][c] = 0.0f;
        }
    }
  }
#pragma unroll
  for (int q = 0; q < CPB; ++q)
#pragma unroll
    for (int c = 0; c < K; ++c) acc[q][c] += (double)lo32[q][c] + (double)cr32[q][c];
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
    const int q = e / K, c = e % K;
    if (q < ncol) {
      double s = red[0][e] + red[1][e] + red[2][e] + red[3][e];
      double* dst = &w.U[(size_t)(j0 + q) * K + c];
      if (accumulate) s += *dst;
      *dst = s;
      if (!isfinite(s)) atomicOr(&w.st->status, ST_NONFINITE);
    }
  }
}

// Partial products of the residual: part[b][r][c] = sum over the columns j of
// chunk b of Q[r][j] * U[j][c], in FP64.  Threads span rows (coalesced).
template <int K>
__global__ __launch_bounds__(256) void resid_part_kernel(Work w, int chunk) {
  if (update_cancelled(w.st)) return;
  const int n = w.n;
  const int r = blockIdx.x * 256 + threadIdx.x;
  const int jb = blockIdx.y * chunk;
  const int je = min(n, jb + chunk);
  __shared__ double su[256 * K];
  double acc[K];
#pragma unroll
  for (int c = 0; c < K; ++c) acc[c] = 0.0;
  const double* __restrict__ Q = w.Q_in;
  for (int j0 = jb; j0 < je; j0 += 256) {
    const int m = min(256, je - j0);
    __syncthreads();
    for (int e = threadIdx.x; e < m * K; e += 256) su[e] = w.U[(size_t)j0 * K + e];
    __syncthreads();
    if (r < n) {
      for (int t = 0; t < m; ++t) {
        const double v = Q[r + (size_t)(j0 + t) * n];
#pragma unroll
        for (int c = 0; c < K; ++c) acc[c] = fma(v, su[t * K + c], acc[c]);
      }
    }
  }
  if (r < n) {
#pragma unroll
    for (int c = 0; c < K; ++c) w.lp_part[((size_t)blockIdx.y * n + r) * K + c] = acc[c];
  }
}

// R = K - sum_b part[b], column-major n x k (leading dimension n).
template <int K>
__global__ __launch_bounds__(256) void resid_reduce_kernel(Work w, int nchunks) {
  if (update_cancelled(w.st)) return;
  const int n = w.n;
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
#pragma unroll
  for (int c = 0; c < K; ++c) {
    double s = 0.0;
    for (int b = 0; b < nchunks; ++b) s += w.lp_part[((size_t)b * n + r) * K + c];
    w.lp_resid[r + (size_t)c * n] = w.K[r + (size_t)c * w.ldk] - s;
  }
}

template <int K, int P>
static hipError_t qtk_lp_launch(const Work& w, hipStream_t s) {
  constexpr int CPB = (K <= 2) ? 8 : 4;
  const int grid = (w.n + CPB - 1) / CPB;
  hipLaunchKernelGGL((qtk_lp_kernel<K, CPB, P>), dim3(grid), dim3(256), 0, s, w, w.K, w.ldk, 0);
  if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
  const int nch = LP_RESID_CHUNKS;
  const int chunk = (w.n + nch - 1) / nch;
  hipLaunchKernelGGL((resid_part_kernel<K>), dim3((w.n + 255) / 256, nch), dim3(256), 0, s, w,
                     chunk);
  if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
  hipLaunchKernelGGL((resid_reduce_kernel<K>), dim3((w.n + 255) / 256), dim3(256), 0, s, w, nch);
  if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
  hipLaunchKernelGGL((qtk_lp_kernel<K, CPB, P>), dim3(grid), dim3(256), 0, s, w,
                     (const double*)w.lp_resid, w.n, 1);
  return hipGetLastError();
}

template <int P>
static hipError_t qtk_lp_dispatch(const Work& w, hipStream_t s) {
  switch (w.k) {
    case 1: return qtk_lp_launch<1, P>(w, s);
    case 2: return qtk_lp_launch<2, P>(w, s);
    case 3: return qtk_lp_launch<3, P>(w, s);
    case 4: return qtk_lp_launch<4, P>(w, s);
    case 5: return qtk_lp_launch<5, P>(w, s);
    case 6: return qtk_lp_launch<6, P>(w, s);
    case 7: return qtk_lp_launch<7, P>(w, s);
    case 8: return qtk_lp_launch<8, P>(w, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_qtk_lp(const Work& w, int prec, hipStream_t s) {
  if (prec == EIG_GEMM_FP32_CORR) return qtk_lp_dispatch<EIG_GEMM_FP32_CORR>(w, s);
  if (prec == EIG_GEMM_BF16X3_CORR) return qtk_lp_dispatch<EIG_GEMM_BF16X3_CORR>(w, s);
  return hipErrorInvalidValue;
}

// ------------------------------------------------------ Q' = Q W (matrix cores)
//
// The operands are split once per update into slice planes (the GEMM below
// only copies them): Ws[s] = slice s of W, column-major like W (k contiguous
// along a column of W); Qs[s] = slice s of Q stored row-major (k contiguous
// along a row of Q), so that both MFMA operands are runs of consecutive k.

template <int P>
struct LpCfg;
template <>
struct LpCfg<EIG_GEMM_FP32_CORR> {
  typedef float T;
  static constexpr int S = 2;    // slices per operand
  static constexpr int BK = 16;  // k per LDS slice (64 bytes of a row)
  static constexpr int RK = 20;  // LDS row length in elements (80 bytes)
};
template <>
struct LpCfg<EIG_GEMM_BF16X3_CORR> {
  typedef unsigned short T;
  static constexpr int S = 3;
  static constexpr int BK = 32;
  static constexpr int RK = 40;
};

// W (n x n column-major FP64) -> S planes of n*n elements, same layout.
// Each thread converts 8 consecutive elements.
template <int P>
__global__ __launch_bounds__(256) void split_w_kernel(const double* __restrict__ W, size_t count,
                                                      void* __restrict__ planes,
                                                      const int32_t* status) {
  if (__builtin_nontemporal_load(status) != 0) return;
  typedef LpCfg<P> Cfg;
  typedef typename Cfg::T T;
  T* out = static_cast<T*>(planes);
  const size_t base = ((size_t)blockIdx.x * 256 + threadIdx.x) * 8;
  if (base >= count) return;
  double x[8];
  if (base + 8 <= count) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double2 v = *reinterpret_cast<const double2*>(W + base + 2 * q);
      x[2 * q] = v.x;
      x[2 * q + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) x[q] = (base + q < count) ? W[base + q] : 0.0;
  }
  T sl[Cfg::S][8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    if constexpr (P == EIG_GEMM_FP32_CORR) {
      split_f32(x[q], sl[0][q], sl[1][q]);
    } else {
      split_bf16x3(x[q], sl[0][q], sl[1][q], sl[2][q]);
    }
  }
#pragma unroll
  for (int s = 0; s < Cfg::S; ++s) {
    T* dst = out + (size_t)s * count + base;
    if (base + 8 <= count && (count & 7) == 0) {
#pragma unroll
      for (int q = 0; q < 8; q += 16 / (int)sizeof(T)) {
        typedef T tv __attribute__((ext_vector_type(16 / sizeof(T))));
        tv v;
#pragma unroll
        for (int e = 0; e < 16 / (int)sizeof(T); ++e) v[e] = sl[s][q + e];
        *reinterpret_cast<tv*>(dst + q) = v;
      }
    } else {
      for (int q = 0; q < 8; ++q)
        if (base + q < count) dst[q] = sl[s][q];
    }
  }
}

// Q (n x n column-major FP64) -> S planes holding the slices of Q row-major:
// plane[s][m * n + k] = slice s of Q[m][k].  64 x 64 tiles through LDS.
template <int P>
__global__ __launch_bounds__(256) void split_qt_kernel(const double* __restrict__ Q, int n,
                                                       void* __restrict__ planes,
                                                       const int32_t* status) {
  if (__builtin_nontemporal_load(status) != 0) return;
  typedef LpCfg<P> Cfg;
  typedef typename Cfg::T T;
  __shared__ double tile[64][65];
  const int m0 = blockIdx.x * 64, k0 = blockIdx.y * 64;
  const int tid = threadIdx.x;
  // load: column k0 + c, rows m0 .. m0 + 63 (coalesced along the column)
  for (int e = tid; e < 64 * 64; e += 256) {
    const int c = e >> 6, r = e & 63;
    const int m = m0 + r, k = k0 + c;
    tile[r][c] = (m < n && k < n) ? Q[(size_t)k * n + m] : 0.0;
  }
  __syncthreads();
  // store: row m0 + r, k = k0 + 8*g .. +8 (16-byte runs of one plane row)
  T* out = static_cast<T*>(planes);
  const size_t nn = (size_t)n * n;
  for (int e = tid; e < 64 * 8; e += 256) {
    const int r = e >> 3, g = e & 7;
    const int m = m0 + r;
    if (m >= n) continue;
    T sl[Cfg::S][8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double x = tile[r][8 * g + q];
      if constexpr (P == EIG_GEMM_FP32_CORR) {
        split_f32(x, sl[0][q], sl[1][q]);
      } else {
        split_bf16x3(x, sl[0][q], sl[1][q], sl[2][q]);
      }
    }
    const int kb = k0 + 8 * g;
#pragma unroll
    for (int s = 0; s < Cfg::S; ++s) {
      T* dst = out + (size_t)s * nn + (size_t)m * n + kb;
      if (kb + 8 <= n && ((n & 7) == 0)) {
#pragma unroll
        for (int q = 0; q < 8; q += 16 / (int)sizeof(T)) {
          typedef T tv __attribute__((ext_vector_type(16 / sizeof(T))));
          tv v;
#pragma unroll
          for (int t = 0; t < 16 / (int)sizeof(T); ++t) v[t] = sl[s][q + t];
          *reinterpret_cast<tv*>(dst + q) = v;
        }
      } else {
        for (int q = 0; q < 8; ++q)
          if (kb + q < n) dst[q] = sl[s][q];
      }
    }
  }
}

constexpr int LBM = 128, LBN = 128, LNT = 256;

__device__ __forceinline__ void lp_tile_of(int bid, int tiles_m, int tiles_n, int* tm, int* tn) {
  // blocks are dealt round-robin to the 8 XCDs: give each XCD a contiguous run
  // of tiles, ordered in groups of 8 tile rows
  const int total = tiles_m * tiles_n;
  const int per = total / 8, rem = total % 8;
  const int x = bid % 8, local = bid / 8;
  const int tile = (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + local;
  const int tpg = 8 * tiles_n;
  const int group = tile / tpg;
  const int first_m = group * 8;
  const int gsz = min(tiles_m - first_m, 8);
  const int in = tile % tpg;
  *tm = first_m + in % gsz;
  *tn = in / gsz;
}

// C (n x n, column-major FP64) = Q W from the slice planes.  Block tile
// 128 x 128, 4 waves of 64 x 64 (4 x 4 MFMA tiles of 16 x 16).  A thread copies
// 16-byte runs of both operands (row t/2 of the tile, half t%2 of the k-slice)
// global -> registers -> LDS with double buffering.
template <int P>
__global__ __launch_bounds__(LNT, 1) void gemm_lp_kernel(int n, const void* __restrict__ Qp,
                                                        const void* __restrict__ Wp,
                                                        double* __restrict__ C,
                                                        const int32_t* status, int tiles) {
  typedef LpCfg<P> Cfg;
  typedef typename Cfg::T T;
  constexpr int S = Cfg::S, BK = Cfg::BK, RK = Cfg::RK;
  constexpr int EPV = 16 / (int)sizeof(T);  // elements per 16-byte run
  constexpr int RUNS = BK / EPV / 2;        // runs per thread per slice plane
  typedef T tv __attribute__((ext_vector_type(EPV)));
  if (__builtin_nontemporal_load(status) != 0) return;
  __shared__ __attribute__((aligned(16))) T As[2][S][LBM][RK];
  __shared__ __attribute__((aligned(16))) T Bs[2][S][LBN][RK];
  int tm, tn;
  lp_tile_of(blockIdx.x, tiles, tiles, &tm, &tn);
  const int m0 = tm * LBM, n0 = tn * LBN;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = (wv & 1) * 64, wn = (wv >> 1) * 64;
  const size_t nn = (size_t)n * n;
  const T* __restrict__ Qs = static_cast<const T*>(Qp);
  const T* __restrict__ Ws = static_cast<const T*>(Wp);
  const int r_row = tid >> 1, r_k = (tid & 1) * (BK / 2);
  const int am = m0 + r_row, bn = n0 + r_row;
  const bool vec = (n % EPV) == 0;
  tv ra[S][RUNS], rb[S][RUNS];

  auto gload = [&](int k0) {
    const bool full_k = vec && (k0 + BK <= n);
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int q = 0; q < RUNS; ++q) {
        const int kk = k0 + r_k + q * EPV;
        if (full_k && am < n) {
          ra[s][q] = *reinterpret_cast<const tv*>(Qs + s * nn + (size_t)am * n + kk);
        } else {
#pragma unroll
          for (int e = 0; e < EPV; ++e)
            ra[s][q][e] = (am < n && kk + e < n) ? Qs[s * nn + (size_t)am * n + kk + e] : T(0);
        }
        if (full_k && bn < n) {
          rb[s][q] = *reinterpret_cast<const tv*>(Ws + s * nn + (size_t)bn * n + kk);
        } else {
#pragma unroll
          for (int e = 0; e < EPV; ++e)
            rb[s][q][e] = (bn < n && kk + e < n) ? Ws[s * nn + (size_t)bn * n + kk + e] : T(0);
        }
      }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int q = 0; q < RUNS; ++q) {
        *reinterpret_cast<tv*>(&As[buf][s][r_row][r_k + q * EPV]) = ra[s][q];
        *reinterpret_cast<tv*>(&Bs[buf][s][r_row][r_k + q * EPV]) = rb[s][q];
      }
  };

  d4 accD[4][4];
  f4 acc[4][4], cross[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      accD[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      acc[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
      cross[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    }

  const int nk = (n + BK - 1) / BK;
  gload(0);
  sstore(0);
  __syncthreads();
  const int fr = lane & 15, fg = lane >> 4;
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * BK);
    if constexpr (P == EIG_GEMM_FP32_CORR) {
      f4 a[2][4], b[2][4];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          a[s][i] = *reinterpret_cast<const f4*>(&As[cur][s][wm + i * 16 + fr][4 * fg]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          b[s][j] = *reinterpret_cast<const f4*>(&Bs[cur][s][wn + j * 16 + fr][4 * fg]);
      }
      // each product sweeps the 16 accumulators, so consecutive MFMAs are
      // independent and issue back to back
#pragma unroll
      for (int t = 0; t < 4; ++t) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            cross[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0][i][t], b[1][j][t], cross[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            cross[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1][i][t], b[0][j][t], cross[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0][i][t], b[0][j][t], acc[i][j], 0, 0, 0);
      }
    } else {
      bf8 a[3][4], b[3][4];
#pragma unroll
      for (int s = 0; s < 3; ++s) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          a[s][i] = *reinterpret_cast<const bf8*>(&As[cur][s][wm + i * 16 + fr][8 * fg]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          b[s][j] = *reinterpret_cast<const bf8*>(&Bs[cur][s][wn + j * 16 + fr][8 * fg]);
      }
      // products b_pa * b_pb, smallest first; each sweeps the 16 accumulators
      // so that consecutive MFMAs are independent
      constexpr int PA[6] = {2, 1, 0, 1, 0, 0}, PB[6] = {0, 1, 2, 0, 1, 0};
#pragma unroll
      for (int p = 0; p < 6; ++p)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[PA[p]][i], b[PB[p]][j], acc[i][j], 0, 0, 0);
    }
    // promote this slice's FP32 partial sums
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int v = 0; v < 4; ++v) accD[i][j][v] += (double)acc[i][j][v];
        acc[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
      }
    if (kt + 1 < nk) sstore(cur ^ 1);
    __syncthreads();
  }
  // epilogue: lane holds rows 4*(l/16) + v (v = 0..3) of column l%16 of each tile
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = n0 + wn + j * 16 + fr;
      if (col >= n) continue;
      double* dst = C + (size_t)col * n;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm + i * 16 + 4 * fg + v;
        double x = accD[i][j][v];
        if (P == EIG_GEMM_FP32_CORR) x += (double)cross[i][j][v];
        if (row < n) dst[row] = x;
      }
    }
}

// The BF16X3 product when n is a multiple of RG_BK: the same slices, products,
// order and promotions as gemm_lp_kernel (bitwise the same C), staged through a
// three-stage LDS ring that the global -> LDS loads (global_load_lds_dwordx4,
// no registers) fill two slices ahead of the MFMAs.  128 x 128 block tile, 8
// waves of 64 x 32 (two waves per SIMD, so one wave's FP64 promotion and waits
// overlap the other's MFMAs).  Each tile row of a plane is 4 chunks of 16 bytes
// (32 k); chunk kc of row r sits at position kc ^ ((r >> 1) & 3), which puts
// the 8 rows an 8-lane group reads at distinct 16-byte bank groups.  Rows past
// n are read from row n - 1 (their outputs are not stored); n % RG_BK == 0
// keeps every k in range.  The loads are not tracked by the compiler's waits:
// before the barrier that opens a slice, each wave waits (vmcnt) until only the
// loads of the later slices are outstanding, and the barrier that closes it
// keeps a stage from being refilled while a wave still reads it.
constexpr int RG_BK = 32;     // k per stage: one MFMA deep
constexpr int RG_STAGES = 3;  // slices kt + 1 and kt + 2 load while slice kt is multiplied
constexpr int RG_NT = 512;

typedef __attribute__((address_space(3))) void* lds_void_ptr;

__global__ __launch_bounds__(RG_NT, 1) void gemm_bf16x3_ring(int n,
                                                           const unsigned short* __restrict__ Qs,
                                                           const unsigned short* __restrict__ Ws,
                                                           double* __restrict__ C,
                                                           const int32_t* status, int tiles) {
  if (__builtin_nontemporal_load(status) != 0) return;
  // [stage][operand: Q, W][plane][tile row][k]: 16-byte chunks, the 4 chunks of a
  // row stored at position kc ^ ((row >> 1) & 3)
  __shared__ __attribute__((aligned(16))) unsigned short L[RG_STAGES][2][3][LBM][RG_BK];
  int tm, tn;
  lp_tile_of(blockIdx.x, tiles, tiles, &tm, &tn);
  const int m0 = tm * LBM, n0 = tn * LBN;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = (wv & 1) * 64, wn = (wv >> 1) * 32;
  const size_t nn = (size_t)n * n;
  // one stage: per operand 3 planes x 128 rows x 4 chunks; instruction i of wave
  // wv loads chunks i * 512 + 64 wv + lane (one plane, 16 rows)
  auto issue = [&](int kt, int stg) {
    const int k0 = kt * RG_BK;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int c0 = i * 512 + wv * 64;
      const int s = c0 >> 9, row0 = (c0 & 511) >> 2;
      const int row = row0 + (lane >> 2), kcs = lane & 3;
      const int kc = kcs ^ ((row >> 1) & 3);
      const int ga = min(m0 + row, n - 1), gb = min(n0 + row, n - 1);
      __builtin_amdgcn_global_load_lds(Qs + s * nn + (size_t)ga * n + k0 + 8 * kc,
                                       (lds_void_ptr)&L[stg][0][s][row0][0], 16, 0, 0);
      __builtin_amdgcn_global_load_lds(Ws + s * nn + (size_t)gb * n + k0 + 8 * kc,
                                       (lds_void_ptr)&L[stg][1][s][row0][0], 16, 0, 0);
    }
  };
  d4 accD[4][2];
  f4 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) accD[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  const int nk = n / RG_BK;
  const int fr = lane & 15, fg = lane >> 4;
  issue(0, 0);
  if (nk > 1) issue(1, 1);
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt % RG_STAGES;
    // stage (kt + 2) % 3 was last read in step kt - 1, before its closing barrier
    if (kt + 2 < nk) {
      issue(kt + 2, (kt + 2) % RG_STAGES);
      asm volatile("s_waitcnt vmcnt(12)" ::: "memory");
    } else if (kt + 1 < nk) {
      asm volatile("s_waitcnt vmcnt(6)" ::: "memory");
    } else {
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    bf8 a[3][4], b[3][2];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = wm + i * 16 + fr;
        a[s][i] = *reinterpret_cast<const bf8*>(&L[cur][0][s][r][8 * (fg ^ ((r >> 1) & 3))]);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int r = wn + j * 16 + fr;
        b[s][j] = *reinterpret_cast<const bf8*>(&L[cur][1][s][r][8 * (fg ^ ((r >> 1) & 3))]);
      }
    }
    // the slice's FP32 partial sums start from zero in the first product
    constexpr int PA[6] = {2, 1, 0, 1, 0, 0}, PB[6] = {0, 1, 2, 0, 1, 0};
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[PA[0]][i], b[PB[0]][j],
                                                            f4{0.0f, 0.0f, 0.0f, 0.0f}, 0, 0, 0);
#pragma unroll
    for (int p = 1; p < 6; ++p)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[PA[p]][i], b[PB[p]][j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) accD[i][j][v] += (double)acc[i][j][v];
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn + j * 16 + fr;
      if (col >= n) continue;
      double* dst = C + (size_t)col * n;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm + i * 16 + 4 * fg + v;
        if (row < n) dst[row] = accD[i][j][v];
      }
    }
}

size_t lp_plane_bytes(int prec, int n) {
  const size_t nn = (size_t)n * n;
  size_t b = 0;
  if (prec == EIG_GEMM_FP32_CORR) b = 2 * nn * sizeof(float);
  if (prec == EIG_GEMM_BF16X3_CORR) b = 3 * nn * sizeof(unsigned short);
  return (b + 255) & ~size_t(255);
}

template <int P>
static hipError_t gemm_lp_launch(const Work& w, void* qplanes, void* wplanes, hipStream_t s) {
  const int n = w.n;
  const size_t nn = (size_t)n * n;
  const int32_t* st = &w.st->status;
  const size_t nthr = (nn + 7) / 8;
  hipLaunchKernelGGL((split_w_kernel<P>), dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, s,
                     (const double*)w.W, nn, wplanes, st);
  if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
  const int t64 = (n + 63) / 64;
  hipLaunchKernelGGL((split_qt_kernel<P>), dim3(t64, t64), dim3(256), 0, s, w.Q_in, n, qplanes,
                     st);
  if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
  const int tiles = (n + LBM - 1) / LBM;
  if (P == EIG_GEMM_BF16X3_CORR && n % RG_BK == 0)
    hipLaunchKernelGGL(gemm_bf16x3_ring, dim3(tiles * tiles), dim3(RG_NT), 0, s, n,
                       static_cast<const unsigned short*>(qplanes),
                       static_cast<const unsigned short*>(wplanes), w.Q_out, st, tiles);
  else
    hipLaunchKernelGGL((gemm_lp_kernel<P>), dim3(tiles * tiles), dim3(LNT), 0, s, n,
                       (const void*)qplanes, (const void*)wplanes, w.Q_out, st, tiles);
  return hipGetLastError();
}

hipError_t launch_gemm_lp(const Work& w, int prec, void* qplanes, void* wplanes, hipStream_t s) {
  if (prec == EIG_GEMM_FP32_CORR) return gemm_lp_launch<EIG_GEMM_FP32_CORR>(w, qplanes, wplanes, s);
  if (prec == EIG_GEMM_BF16X3_CORR)
    return gemm_lp_launch<EIG_GEMM_BF16X3_CORR>(w, qplanes, wplanes, s);
  return hipErrorInvalidValue;
}

}  // namespace eigupd
