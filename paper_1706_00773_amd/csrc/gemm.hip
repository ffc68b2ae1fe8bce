// gemm.hip -- C = A B in FP64 on the CDNA4 matrix cores (the back-transform
// Q' = Q W of Sec. 2.4, eq. (10): 2 n^3 flops, the dominant step).
//
// v_mfma_f64_16x16x4_f64: per wave, A fragment 16x4 (lane l holds A[l%16][l/16]),
// B fragment 4x16 (lane l holds B[l/16][l%16]), accumulator 16x16 (lane l holds
// rows l/16 + 4v, v = 0..3, of column l%16).
//
// Tiling: 128x128 block tile, 16-deep k slices, 256 threads = 4 waves in a 2x2
// arrangement, each wave a 64x64 sub-tile = 4x4 MFMA tiles (64 doubles of
// accumulator per lane).  Slices are staged global -> registers -> LDS with two
// register sets and two LDS buffers: while the MFMAs consume slice s from LDS,
// slice s + 1 waits in registers to be stored and the global loads of slice
// s + 2 are in flight (two slices of latency hidden), one barrier per slice.  Block ids are remapped so
// that the blocks resident on one XCD (blocks are dealt round-robin to the 8
// XCDs) cover one compact group of 8 tile rows, sharing its A panel and the B
// panels in that XCD's L2.  LDS rows are padded to 144 doubles (288 dwords, an
// odd multiple of 32 banks), so the four k-rows an MFMA fragment read touches
// fall in alternating bank halves and the fragment reads are conflict free.
#include "common.h"

namespace eigupd {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int GBM = 128, GBN = 128, GBK = 16, GPAD = 16, GNT = 256;
constexpr int GGROUP = 8;

__device__ __forceinline__ void tile_of(int bid, int tiles_m, int tiles_n, int* tm, int* tn) {
  const int total = tiles_m * tiles_n;
  const int per = total / 8, rem = total % 8;
  const int x = bid % 8, local = bid / 8;
  const int tile = (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + local;
  const int tpg = GGROUP * tiles_n;
  const int group = tile / tpg;
  const int first_m = group * GGROUP;
  const int gsz = min(tiles_m - first_m, GGROUP);
  const int in = tile % tpg;
  *tm = first_m + in % gsz;
  *tn = in / gsz;
}

// One BT x BT tile (tm, tn) of C = A B.  Four waves in a 2 x 2 arrangement, each
// a (BT/2) x (BT/2) sub-tile of 16 x 16 MFMA tiles.  A thread stages BT/16
// doubles of the A slice (pairs of rows 32 apart in one k-column) and BT/16 of
// the B slice (consecutive k of one column of B).  Every tile size runs the
// same k-slices in the same order, so C is bitwise the same for any BT.
// ACC: C += A B instead of C = A B.  Src supplies, for k-slice s, the operands
// and the slice's offset and extent in them (one matrix pair, or segments of
// several pairs summed into one C); kg is the slice's offset in the summed k.
struct PlainSrc {
  const double* A;
  const double* B;
  int lda, ldb, K;
  __device__ __forceinline__ int slices() const { return (K + GBK - 1) / GBK; }
  __device__ __forceinline__ void at(int kg, const double* __restrict__& a, int& la,
                                     const double* __restrict__& b, int& lb,
                                     int& k0, int& kd) const {
    a = A;
    la = lda;
    b = B;
    lb = ldb;
    k0 = kg;
    kd = K;
  }
};

// Segments are visited in increasing slice order (the tile asks for slices
// 0, 1, 2, ...), so a cursor loads the next segment's operands only when the
// slice index crosses a segment end.
struct SegSrc {
  const GemmSegDesc& d;
  int i = -1, s0 = 0, s1 = 0;  // current segment and its slices [s0, s1)
  const double* A = nullptr;
  const double* B = nullptr;
  int lda = 0, ldb = 0, K = 0;
  __device__ __forceinline__ int slices() const { return d.send[d.nseg - 1]; }
  __device__ __forceinline__ void at(int kg, const double* __restrict__& a, int& la,
                                     const double* __restrict__& b, int& lb, int& k0, int& kd) {
    const int s = kg / GBK;
    while (s >= s1 && i + 1 < d.nseg) {
      ++i;
      s0 = s1;
      s1 = d.send[i];
      A = d.A[i];
      B = d.B[i];
      lda = d.lda[i];
      ldb = d.ldb[i];
      K = d.K[i];
    }
    a = A;
    la = lda;
    b = B;
    lb = ldb;
    k0 = (s - s0) * GBK;
    kd = K;
  }
};

template <int BT, bool ACC, typename Src>
__device__ __forceinline__ void dgemm_tile_src(int M, int N, Src src,
                                               double* __restrict__ C, int ldc, int tm, int tn,
                                               int vec) {
  constexpr int WT = BT / 2;          // wave sub-tile
  constexpr int FT = WT / 16;         // MFMA tiles per wave side
  constexpr int AQ = BT / 32;         // A row pairs per thread
  constexpr int TPC = GNT / BT;       // threads per B column
  constexpr int KPT = GBK / TPC;      // k values per thread of a B column
  __shared__ double As[2][GBK][BT + GPAD];
  __shared__ double Bs[2][GBK][BT + GPAD];
  const int m0 = tm * BT, n0 = tn * BT;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = (wv & 1) * WT, wn = (wv >> 1) * WT;
  // A: column k0+a_k, rows m0+a_m+32q .. +2: each group of 16 lanes writes one
  // LDS row in 16-byte pairs, so the stores do not collide
  const int a_k = tid >> 4, a_m = (tid & 15) * 2;
  const int b_n = tid / TPC, b_k = (tid % TPC) * KPT;  // B: column n0+b_n, rows k0+b_k ..
  const bool full_m = vec && (m0 + BT <= M), full_n = vec && (n0 + BT <= N);
  double ra0[2 * AQ], rb0[KPT], ra1[2 * AQ], rb1[KPT];

  auto gload = [&](int kg, double (&ra)[2 * AQ], double (&rb)[KPT]) {
    const double* __restrict__ A;
    const double* __restrict__ B;
    int lda, ldb, k0, Kd;
    src.at(kg, A, lda, B, ldb, k0, Kd);
    const bool full_k = (k0 + GBK <= Kd);
    const int ka = k0 + a_k;
    if (full_m && full_k) {
#pragma unroll
      for (int q = 0; q < AQ; ++q) {
        const double2 v = *reinterpret_cast<const double2*>(A + (size_t)ka * lda + m0 + a_m + 32 * q);
        ra[2 * q] = v.x;
        ra[2 * q + 1] = v.y;
      }
    } else {
#pragma unroll
      for (int q = 0; q < 2 * AQ; ++q) {
        const int r = m0 + a_m + 32 * (q >> 1) + (q & 1);
        ra[q] = (r < M && ka < Kd) ? A[(size_t)ka * lda + r] : 0.0;
      }
    }
    const int nb = n0 + b_n;
    if (full_n && full_k) {
      const double2* src = reinterpret_cast<const double2*>(B + (size_t)nb * ldb + k0 + b_k);
#pragma unroll
      for (int q = 0; q < KPT / 2; ++q) {
        const double2 v = src[q];
        rb[2 * q] = v.x;
        rb[2 * q + 1] = v.y;
      }
    } else {
#pragma unroll
      for (int q = 0; q < KPT; ++q) {
        const int kk = k0 + b_k + q;
        rb[q] = (nb < N && kk < Kd) ? B[(size_t)nb * ldb + kk] : 0.0;
      }
    }
  };
  auto sstore = [&](int buf, const double (&ra)[2 * AQ], const double (&rb)[KPT]) {
#pragma unroll
    for (int q = 0; q < AQ; ++q)
      *reinterpret_cast<double2*>(&As[buf][a_k][a_m + 32 * q]) = double2{ra[2 * q], ra[2 * q + 1]};
#pragma unroll
    for (int q = 0; q < KPT; ++q) Bs[buf][b_k + q][b_n] = rb[q];
  };

  d4 acc[FT][FT];
#pragma unroll
  for (int i = 0; i < FT; ++i)
#pragma unroll
    for (int j = 0; j < FT; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  const int nk = src.slices();
  const int fr = lane & 15, fk = lane >> 4;
  auto compute = [&](int cur) {
#pragma unroll
    for (int ks = 0; ks < GBK / 4; ++ks) {
      const int kr = ks * 4 + fk;
      double a[FT], b[FT];
#pragma unroll
      for (int i = 0; i < FT; ++i) a[i] = As[cur][kr][wm + i * 16 + fr];
#pragma unroll
      for (int j = 0; j < FT; ++j) b[j] = Bs[cur][kr][wn + j * 16 + fr];
#pragma unroll
      for (int i = 0; i < FT; ++i)
#pragma unroll
        for (int j = 0; j < FT; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  };
  gload(0, ra0, rb0);
  sstore(0, ra0, rb0);
  if (nk > 1) gload(GBK, ra1, rb1);
  __syncthreads();
  // slice s sits in register set s & 1 until it is stored; two slices in flight
  int kt = 0;
  for (; kt + 1 < nk; kt += 2) {
    if (kt + 2 < nk) gload((kt + 2) * GBK, ra0, rb0);
    compute(0);
    sstore(1, ra1, rb1);
    __syncthreads();
    if (kt + 3 < nk) gload((kt + 3) * GBK, ra1, rb1);
    compute(1);
    if (kt + 2 < nk) sstore(0, ra0, rb0);
    __syncthreads();
  }
  if (kt < nk) compute(0);
  // epilogue: lane holds rows l/16 + 4v of column l%16 of each 16x16 tile; for a
  // fixed v the wave writes 4 consecutive rows of 16 columns
#pragma unroll
  for (int i = 0; i < FT; ++i)
#pragma unroll
    for (int j = 0; j < FT; ++j) {
      const int col = n0 + wn + j * 16 + fr;
      if (col < N) {
        double* dst = C + (size_t)col * ldc;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = m0 + wm + i * 16 + fk + 4 * v;
          if (row < M) {
            if constexpr (ACC)
              dst[row] += acc[i][j][v];
            else
              dst[row] = acc[i][j][v];
          }
        }
      }
    }
}

template <int BT, bool ACC = false>
__device__ __forceinline__ void dgemm_tile(int M, int N, int Kd, const double* __restrict__ A,
                                           int lda, const double* __restrict__ B, int ldb,
                                           double* __restrict__ C, int ldc, int tm, int tn,
                                           int vec) {
  dgemm_tile_src<BT, ACC>(M, N, PlainSrc{A, B, lda, ldb, Kd}, C, ldc, tm, tn, vec);
}

__global__ __launch_bounds__(GNT, 2) void dgemm_kernel(int M, int N, int Kd,
                                                       const double* __restrict__ A, int lda,
                                                       const double* __restrict__ B, int ldb,
                                                       double* __restrict__ C, int ldc,
                                                       const int32_t* status, int tiles_m,
                                                       int tiles_n, int vec) {
  if (__builtin_nontemporal_load(status) != 0) return;
  int tm, tn;
  tile_of(blockIdx.x, tiles_m, tiles_n, &tm, &tn);
  dgemm_tile<GBM>(M, N, Kd, A, lda, B, ldb, C, ldc, tm, tn, vec);
}

// Grouped Q' = Q W over several instances: block b is tile b - prefix[i] of
// instance i (tiles in groups of GGROUP tile rows, column by column).
template <int BT>
__global__ __launch_bounds__(GNT, 2) void dgemm_group(const GemmDesc* __restrict__ d,
                                                      const int* __restrict__ prefix, int ninst) {
  int lo = 0, hi = ninst - 1;
  const int b = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  const GemmDesc& g = d[lo];
  if (__builtin_nontemporal_load(g.status) != 0) return;
  const int t = b - prefix[lo];
  const int tiles = (g.n + BT - 1) / BT;
  const int tpg = GGROUP * tiles;
  const int first_m = (t / tpg) * GGROUP;
  const int gsz = min(tiles - first_m, GGROUP);
  const int in = t % tpg;
  dgemm_tile<BT>(g.n, g.n, g.n, g.A, g.n, g.B, g.n, g.C, g.n, first_m + in % gsz, in / gsz, g.vec);
}

// Products of general shapes from device-built descriptors: block b is tile
// b - prefix[i] of instance i, tiles ordered down the columns of C.  Skipped on
// the device when *skip != 0.
template <bool ACC, int BT>
__global__ __launch_bounds__(GNT, 2) void dgemm_desc(const GemmDescG* __restrict__ d,
                                                     const int* __restrict__ prefix, int ninst,
                                                     const int32_t* skip) {
  if (__builtin_nontemporal_load(skip) != 0) return;
  int lo = 0, hi = ninst - 1;
  const int b = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  const GemmDescG& g = d[lo];
  if (g.M <= 0 || g.N <= 0 || g.K <= 0) return;  // an empty instance
  const int t = b - prefix[lo];
  dgemm_tile<BT, ACC>(g.M, g.N, g.K, g.A, g.lda, g.B, g.ldb, g.C, g.ldc, t % g.tiles_m,
                      t / g.tiles_m, g.vec);
}

// Segmented products C = sum_i A_i B_i from device-built descriptors (block b is
// tile b - prefix[i] of instance i); skipped on the device when *skip != 0.
__global__ __launch_bounds__(GNT, 2) void dgemm_seg(const GemmSegDesc* __restrict__ d,
                                                    const int* __restrict__ prefix, int ninst,
                                                    const int32_t* skip) {
  if (__builtin_nontemporal_load(skip) != 0) return;
  int lo = 0, hi = ninst - 1;
  const int b = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  const GemmSegDesc& g = d[lo];
  if (g.M <= 0 || g.N <= 0 || g.nseg <= 0) return;
  const int t = b - prefix[lo];
  dgemm_tile_src<GBM, false>(g.M, g.N, SegSrc{g}, g.C, g.ldc, t % g.tiles_m, t / g.tiles_m,
                             g.vec);
}

hipError_t launch_dgemm_seg(const GemmSegDesc* d, const int* prefix, int ninst, int blocks,
                            const int32_t* skip, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(dgemm_seg, dim3(blocks), dim3(GNT), 0, s, d, prefix, ninst, skip);
  return hipGetLastError();
}

hipError_t launch_dgemm_desc(bool acc, int bt, const GemmDescG* d, const int* prefix, int ninst,
                             int blocks, const int32_t* skip, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  if (bt == 128 && acc)
    hipLaunchKernelGGL((dgemm_desc<true, 128>), dim3(blocks), dim3(GNT), 0, s, d, prefix, ninst,
                       skip);
  else if (bt == 128)
    hipLaunchKernelGGL((dgemm_desc<false, 128>), dim3(blocks), dim3(GNT), 0, s, d, prefix, ninst,
                       skip);
  else if (bt == 64 && !acc)
    hipLaunchKernelGGL((dgemm_desc<false, 64>), dim3(blocks), dim3(GNT), 0, s, d, prefix, ninst,
                       skip);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

int gemm_tiles(int n, int bt) {
  const int t = (n + bt - 1) / bt;
  return t * t;
}

hipError_t launch_dgemm_group(int bt, const GemmDesc* d, const int* prefix, int ninst, int blocks,
                              hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  if (bt == 128)
    hipLaunchKernelGGL((dgemm_group<128>), dim3(blocks), dim3(GNT), 0, s, d, prefix, ninst);
  else if (bt == 64)
    hipLaunchKernelGGL((dgemm_group<64>), dim3(blocks), dim3(GNT), 0, s, d, prefix, ninst);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_dgemm(int M, int N, int Kd, const double* A, int lda, const double* B, int ldb,
                        double* C, int ldc, const int32_t* status, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  // 16-byte vector loads and stores need every column start 16-byte aligned
  const int vec = !((lda & 1) || (ldb & 1) || (ldc & 1) || ((uintptr_t)A & 15) ||
                    ((uintptr_t)B & 15) || ((uintptr_t)C & 15));
  const int tiles_m = (M + GBM - 1) / GBM, tiles_n = (N + GBN - 1) / GBN;
  hipLaunchKernelGGL(dgemm_kernel, dim3(tiles_m * tiles_n), dim3(GNT), 0, s, M, N, Kd, A, lda,
                     B, ldb, C, ldc, status, tiles_m, tiles_n, vec);
  return hipGetLastError();
}

}  // namespace eigupd
