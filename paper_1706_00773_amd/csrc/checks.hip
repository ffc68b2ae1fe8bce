// checks.hip -- the device checks of EIG_DEBUG_CHECKS, run after an update and
// before its commit.  A failed check raises the sticky ST_CHECK bit: nothing
// is committed and the next eig_query reports EIG_ECHECK.
//
// What is checked (ahat = max|lambda| + ||U||_F^2 >= ||A'||_2, bwd = the
// deflation's backward-error bound):
//   - the new eigenvalues are ascending;
//   - each lies in its Courant-Weyl window [lambda_{i-q}, lambda_{i+p}]
//     (Sec. 2.2; the outer bounds past the ends), within 8 eps ahat + bwd;
//   - trace: sum lambda' - sum lambda = sum_c sigma_c ||U_c||^2 within
//     16 n eps ahat + n bwd;
//   - 8 sampled columns w of W (when W is whole): the residual of
//     (diag(lambda) + U Sigma U^T) w = lambda' w (the eigenproblem in the Q
//     basis, eq. (10)) at most 1e-9 ahat + 2 bwd, and their Gram matrix within
//     1e-9 of I;
//   - the same 8 columns of Q' = Q W: Gram matrix within tol_q of I (1e-9 for
//     the FP64 product, the reduced modes' bound otherwise).
#include "common.h"

namespace eigupd {

constexpr int CHK_NT = 256;
constexpr int CHK_COLS = 8;
constexpr double CHK_EPS = 1.1102230246251565e-16;

__device__ __forceinline__ double chk_block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < CHK_NT / 64; ++q) t += sh[q];
  return t;
}

// The sampled column t of CHK_COLS (distinct when n >= CHK_COLS).
__device__ __forceinline__ int chk_col(int n, int t) {
  return (n >= CHK_COLS) ? (int)(((long long)(n - 1) * t) / (CHK_COLS - 1)) : min(t, n - 1);
}

template <int K>
__global__ __launch_bounds__(CHK_NT) void debug_check_kernel(Work w, int check_w, int check_q,
                                                            double tol_q) {
  __shared__ double sh[CHK_NT / 64];
  __shared__ int s_bad;
  if (update_cancelled(w.st)) return;
  const int n = w.n;
  const DevInfo* info = w.info;
  const double ahat = info->ahat, bwd = info->bwd;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  bool bad = false;
  if (blockIdx.x == CHK_COLS) {
    // eigenvalues: order, windows, trace.  The outer bounds past the ends are
    // lambda_1 - sum_{sigma=-1} ||U_c||^2 and lambda_n + sum_{sigma=+1} ||U_c||^2.
    const int p = info->p, q = info->q;
    const double t = 8.0 * CHK_EPS * ahat + bwd;
    double dl = 0.0, pos = 0.0, neg = 0.0;
    for (int i = threadIdx.x; i < n; i += CHK_NT) {
      dl += w.lam_fin[i] - w.lam_in[i];
#pragma unroll
      for (int c = 0; c < K; ++c) {
        const double u = w.U[(size_t)i * K + c];
        if ((w.sig_pos_mask >> c) & 1)
          pos += u * u;
        else
          neg += u * u;
      }
    }
    dl = chk_block_sum(dl, sh);
    pos = chk_block_sum(pos, sh);
    neg = chk_block_sum(neg, sh);
    if (threadIdx.x == 0 && !(fabs(dl - (pos - neg)) <= 16.0 * n * CHK_EPS * ahat + n * bwd))
      bad = true;
    const double lo_end = w.lam_in[0] - neg, hi_end = w.lam_in[n - 1] + pos;
    for (int i = threadIdx.x; i < n; i += CHK_NT) {
      const double x = w.lam_fin[i];
      if (i + 1 < n && !(w.lam_fin[i + 1] >= x)) bad = true;
      const double lo = (i - q >= 0) ? w.lam_in[i - q] : lo_end;
      const double hi = (i + p < n) ? w.lam_in[i + p] : hi_end;
      if (!(x >= lo - t && x <= hi + t)) bad = true;
    }
  } else {
    const int t = blockIdx.x;
    const int pt = chk_col(n, t);
    if (check_w) {
      const double* wc = w.W + (size_t)pt * n;
      double z[K];
#pragma unroll
      for (int c = 0; c < K; ++c) {
        double a = 0.0;
        for (int j = threadIdx.x; j < n; j += CHK_NT) a += w.U[(size_t)j * K + c] * wc[j];
        z[c] = chk_block_sum(a, sh) * (((w.sig_pos_mask >> c) & 1) ? 1.0 : -1.0);
      }
      const double lp = w.lam_fin[pt];
      double r2 = 0.0;
      for (int j = threadIdx.x; j < n; j += CHK_NT) {
        double r = (w.lam_in[j] - lp) * wc[j];
#pragma unroll
        for (int c = 0; c < K; ++c) r += w.U[(size_t)j * K + c] * z[c];
        r2 += r * r;
      }
      r2 = chk_block_sum(r2, sh);
      if (threadIdx.x == 0 && !(sqrt(r2) <= 1e-9 * ahat + 2.0 * bwd)) bad = true;
      for (int b = t; b < CHK_COLS; ++b) {
        const int pb = chk_col(n, b);
        if (b > t && pb == pt) continue;
        const double* wb = w.W + (size_t)pb * n;
        double g = 0.0;
        for (int j = threadIdx.x; j < n; j += CHK_NT) g += wc[j] * wb[j];
        g = chk_block_sum(g, sh);
        if (threadIdx.x == 0 && !(fabs(g - ((b == t) ? 1.0 : 0.0)) <= 1e-9)) bad = true;
      }
    }
    if (check_q) {
      const double* qc = w.Q_out + (size_t)pt * n;
      for (int b = t; b < CHK_COLS; ++b) {
        const int pb = chk_col(n, b);
        if (b > t && pb == pt) continue;
        const double* qb = w.Q_out + (size_t)pb * n;
        double g = 0.0;
        for (int j = threadIdx.x; j < n; j += CHK_NT) g += qc[j] * qb[j];
        g = chk_block_sum(g, sh);
        if (threadIdx.x == 0 && !(fabs(g - ((b == t) ? 1.0 : 0.0)) <= tol_q)) bad = true;
      }
    }
  }
  if (bad) atomicOr(&s_bad, 1);
  __syncthreads();
  if (threadIdx.x == 0 && s_bad) atomicOr(&w.st->status, ST_CHECK);
}

template <int K>
static hipError_t debug_check_launch(const Work& w, int check_w, int check_q, double tol_q,
                                     hipStream_t s) {
  hipLaunchKernelGGL((debug_check_kernel<K>), dim3(CHK_COLS + 1), dim3(CHK_NT), 0, s, w,
                     check_w, check_q, tol_q);
  return hipGetLastError();
}

hipError_t launch_debug_checks(const Work& w, bool check_w, bool check_q, double tol_q,
                               hipStream_t s) {
  EIGUPD_SWITCH_K(w.k, debug_check_launch, w, check_w ? 1 : 0, check_q ? 1 : 0, tol_q, s)
}

}  // namespace eigupd
