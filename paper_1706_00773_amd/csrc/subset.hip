// subset.hip -- V = Q W for the few eigenvectors of eig_update_interval
// (Sec. 2.1: an interval of eigenvalues from the counts alone; Sec. 3: a subset
// of eigenvectors costs far less than a whole decomposition).
#include "common.h"

namespace eigupd {

// ---------------------------------------------------------------------------
// V = Q W for a skinny W (n x m, m <= SK_MMAX): the subset product of
// eig_update_interval.  With m far below a tile width, the MFMA GEMM runs
// n/128 blocks that each stream all of K; this product is instead bound by
// reading Q once (8 n^2 bytes, 2 n^2 m flops on the vector units).  Split k:
// block (row block rb, k split s, column chunk cb) forms the 512 x MC partial
// sums of rows rb*512.., k in split s, columns cb*MC..; each thread owns two
// consecutive rows (one 16-byte load of Q per k) and the block's slice of W
// sits in LDS.  A second kernel adds the splits in order (deterministic).  The
// partial sums need ks * m * n doubles of workspace.  Above 32 columns each
// 32-column chunk streams Q again; up to 128 columns that still beats the
// GEMM's n/128 blocks.
// ---------------------------------------------------------------------------
constexpr int SK_NT = 256, SK_RB = 2 * SK_NT, SK_KC = 128, SK_MMAX = 128;

template <int MC>
__global__ __launch_bounds__(SK_NT) void skinny_part(int n, int m, const double* __restrict__ Q,
                                                     int ldq, const double* __restrict__ W,
                                                     int ldw, double* __restrict__ part,
                                                     const int32_t* status) {
  if (__builtin_nontemporal_load(status) != 0) return;
  constexpr int LDW = MC + 2;  // 16-byte aligned LDS rows
  __shared__ __attribute__((aligned(16))) double sw[SK_KC][LDW];
  const int s = blockIdx.y, c0 = blockIdx.z * MC;
  const int k0 = s * SK_KC, kn = min(SK_KC, n - k0);
  const int mc = min(MC, m - c0);
  for (int e = threadIdx.x; e < SK_KC * MC; e += SK_NT) {
    const int j = e % SK_KC, c = e / SK_KC;
    sw[j][c] = (j < kn && c < mc) ? W[(size_t)(c0 + c) * ldw + k0 + j] : 0.0;
  }
  __syncthreads();
  const int r = blockIdx.x * SK_RB + 2 * threadIdx.x;
  if (r >= n) return;  // n is even: rows r and r + 1 are both in range
  double a0[MC], a1[MC];
#pragma unroll
  for (int c = 0; c < MC; ++c) a0[c] = a1[c] = 0.0;
  const double* __restrict__ q = Q + (size_t)k0 * ldq + r;
#pragma unroll 4
  for (int j = 0; j < kn; ++j) {
    const double2 v = *reinterpret_cast<const double2*>(q + (size_t)j * ldq);
#pragma unroll
    for (int c = 0; c < MC; ++c) {
      a0[c] = fma(v.x, sw[j][c], a0[c]);
      a1[c] = fma(v.y, sw[j][c], a1[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < MC; ++c) {
    if (c < mc) {
      double* dst = part + ((size_t)s * m + c0 + c) * n + r;
      dst[0] = a0[c];
      dst[1] = a1[c];
    }
  }
}

__global__ __launch_bounds__(256) void skinny_reduce(int n, int m, int ks,
                                                     const double* __restrict__ part,
                                                     double* __restrict__ V, int ldv,
                                                     const int32_t* status) {
  if (__builtin_nontemporal_load(status) != 0) return;
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (size_t)n * m) return;
  const int r = (int)(e % n), c = (int)(e / n);
  double v = 0.0;
  for (int s = 0; s < ks; ++s) v += part[((size_t)s * m + c) * n + r];
  V[(size_t)c * ldv + r] = v;
}

size_t skinny_workspace(int n, int m) {
  const int ks = (n + SK_KC - 1) / SK_KC;
  return (size_t)ks * m * n * sizeof(double);
}

bool skinny_applies(int n, int m, const double* Q, int ldq) {
  return m >= 1 && m <= SK_MMAX && !(n & 1) && !(ldq & 1) && !((uintptr_t)Q & 15);
}

hipError_t launch_skinny_qw(int n, int m, const double* Q, int ldq, const double* W, int ldw,
                            double* V, int ldv, double* part, const int32_t* status,
                            hipStream_t s) {
  if (!skinny_applies(n, m, Q, ldq)) return hipErrorInvalidValue;
  const int ks = (n + SK_KC - 1) / SK_KC, rb = (n + SK_RB - 1) / SK_RB;
  if (m <= 8) {
    hipLaunchKernelGGL((skinny_part<8>), dim3(rb, ks, (m + 7) / 8), dim3(SK_NT), 0, s, n, m, Q,
                       ldq, W, ldw, part, status);
  } else if (m <= 16) {
    hipLaunchKernelGGL((skinny_part<16>), dim3(rb, ks, (m + 15) / 16), dim3(SK_NT), 0, s, n, m,
                       Q, ldq, W, ldw, part, status);
  } else {
    hipLaunchKernelGGL((skinny_part<32>), dim3(rb, ks, (m + 31) / 32), dim3(SK_NT), 0, s, n, m,
                       Q, ldq, W, ldw, part, status);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t total = (size_t)n * m;
  hipLaunchKernelGGL(skinny_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, n, m,
                     ks, part, V, ldv, status);
  return hipGetLastError();
}

}  // namespace eigupd
