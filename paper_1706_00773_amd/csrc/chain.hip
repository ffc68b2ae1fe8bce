// chain.hip -- the secular Sturm chain of Sec. 2.2 (eqs. (4)-(9)) as an
// alternative eigenvalue counter.
//
// The reduced secular function f_0(x) = 1 - sum_s alpha_s / (x - d_s) (eq. (4),
// simple poles d_s ascending) times pi_0(x) = prod_s (x - d_s) is the polynomial
// p_0 whose zeros are the eigenvalues of the reduced problem.  Each member of
// its Sturm sequence is kept in the same secular form,
//   p_m = f_m pi_m,  f_m(x) = c_m - sum_{j < N-m} alpha^m_j / (x - d_j),
//   pi_m(x) = prod_{j < N-m} (x - d_j),
// so member m is N - m + 1 numbers:
//   m = 1 (eq. (6)): mu_j = 1 - sum_{i != j} (alpha_i + alpha_j) / (d_j - d_i),
//          c_1 = sum mu_j, alpha^1_j = (d_{N-1} - d_j) mu_j;
//   m >= 2, the secular long division p_m = -p_{m-2} + A_m (x - B_m) p_{m-1}
//          with e1 = d_{N-m}, e2 = d_{N-m+1}, S1^l = sum alpha^l, S2^l = sum alpha^l d:
//          A_m = c_{m-2} / c_{m-1},
//          B_m = e2 + S1^{m-2} / c_{m-2} - S1^{m-1} / c_{m-1}  (the printed B_m with
//          its sign corrected),
//          alpha^m_j = -alpha^{m-2}_j (d_j - e1)(d_j - e2) + A_m (d_j - B_m) alpha^{m-1}_j (d_j - e1),
//          c_m = -(c_{m-2} e1 e2 + S1^{m-2} (e1 + e2) - S2^{m-2})
//                + A_m (c_{m-1} B_m e1 + S1^{m-1} (B_m + e1) - S2^{m-1}).
// The construction stops at the first c_m that is not positive (the chain is
// then partial; its positive c's bound the number of zeros from below).  Zeros
// below x: V(-inf) - V(x), V the sign changes of p_0(x) .. p_M(x); at -inf the
// sign of p_m is (-1)^(N-m) sign(c_m).
//
// Known zeros xi_p are divided out first (eqs. (7)-(9)): with the p-th lowest
// pole removed for the p-th zero, the residues on the remaining poles become
// beta_j = alpha_j prod_p (d_j - d_p) / (d_j - xi_p).
//
// The build is serial in m (one block, one block reduction per level); the
// residues and level 1 are O(N^2), one wave per pole.
#include "common.h"
#include "smallmat.h"

namespace eigupd {

constexpr int CNT = 1024;   // chain build block
constexpr int CHUNK = 4096; // member signs held in LDS at a time by the count kernel

// Residues of eq. (2) for simple poles: with G = sum_{l != s} u_l u_l^T / (d_l - d_s)
// and H = Sigma + G (= Sigma - T_s), alpha_s = det(Sigma) u_s^T adj(H) u_s
// = det(Sigma) sum_m (v_m^T u_s)^2 prod_{l != m} theta_l for H = V diag(theta) V^T
// (no division, so a singular H needs no special case).
template <int K>
__global__ __launch_bounds__(256) void residue_kernel(Work w, double* __restrict__ alpha) {
  constexpr int NS = Sym<K>::NS;
  const int n_d = w.info->n_d;
  const int lane = threadIdx.x & 63;
  // one wave per pole s; the lanes stride the other poles (coalesced reads)
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= n_d) return;
  const double ds = w.rd[s];
  double H[NS];
#pragma unroll
  for (int e = 0; e < NS; ++e) H[e] = 0.0;
  for (int l = lane; l < n_d; l += 64) {
    if (l == s) continue;
    const double r = 1.0 / (w.rd[l] - ds);
    double u[K];
#pragma unroll
    for (int c = 0; c < K; ++c) u[c] = w.ru[(size_t)l * K + c];
#pragma unroll
    for (int a = 0; a < K; ++a) {
      const double ua = u[a] * r;
#pragma unroll
      for (int b = a; b < K; ++b) H[Sym<K>::at(a, b)] = fma(ua, u[b], H[Sym<K>::at(a, b)]);
    }
  }
#pragma unroll
  for (int e = 0; e < NS; ++e) H[e] = wave_sum(H[e]);
  if (lane != 0) return;
  double detsig = 1.0;
#pragma unroll
  for (int c = 0; c < K; ++c) {
    const double sg = ((w.sig_pos_mask >> c) & 1) ? 1.0 : -1.0;
    H[Sym<K>::at(c, c)] += sg;
    detsig *= sg;
  }
  double V[K][K];
  jacobi_eig<K, true>(H, V);
  double us[K];
#pragma unroll
  for (int c = 0; c < K; ++c) us[c] = w.ru[(size_t)s * K + c];
  double acc = 0.0;
#pragma unroll
  for (int m = 0; m < K; ++m) {
    double p = 0.0;
#pragma unroll
    for (int c = 0; c < K; ++c) p = fma(V[c][m], us[c], p);
    double prod = p * p;
#pragma unroll
    for (int l = 0; l < K; ++l)
      if (l != m) prod *= H[Sym<K>::at(l, l)];
    acc += prod;
  }
  alpha[s] = detsig * acc;
}

// Found-zero deflation (eq. (9)): beta_j for the poles j >= s that remain.  Flags
// bad input (zeros not ascending, or a zero on a remaining pole) in *bad.
__global__ __launch_bounds__(256) void chain_deflate_kernel(const double* __restrict__ d, int n,
                                                            const double* __restrict__ xi, int s,
                                                            double* __restrict__ alpha, int* bad) {
  if (blockIdx.x == 0)
    for (int t = threadIdx.x; t + 1 < s; t += blockDim.x)
      if (!(xi[t] < xi[t + 1])) atomicOr(bad, 1);
  const int j = s + blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double dj = d[j];
  double b = alpha[j];
  for (int p = 0; p < s; ++p) {
    const double den = dj - xi[p];
    if (den == 0.0) atomicOr(bad, 1);
    b = b * (dj - d[p]) / den;
  }
  alpha[j] = b;
}

// Level 1: mu_j = 1 - sum_{i != j} (alpha_i + alpha_j) / (d_j - d_i); one wave per j.
__global__ __launch_bounds__(256) void chain_mu_kernel(const double* __restrict__ d,
                                                       const double* __restrict__ alpha, int n,
                                                       double* __restrict__ mu) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n) return;
  const double dj = d[j], aj = alpha[j];
  double acc = 0.0;
  for (int i = lane; i < n; i += 64) {
    if (i == j) continue;
    acc += (alpha[i] + aj) / (dj - d[i]);
  }
  acc = wave_sum(acc);
  if (lane == 0) mu[j] = 1.0 - acc;
}

// Offset of member m in the triangular level storage (member m has n - m entries).
__device__ __host__ __forceinline__ size_t level_off(int n, int m) {
  return (size_t)m * n - (size_t)m * (m - 1) / 2;
}

struct ChainOut {
  int levels;    // members built
  int complete;  // all n + 1 members with every c positive
};

// The serial build, members 0 .. levels-1, one block.  lv holds the members
// (level_off layout), c the leading constants.  mu from chain_mu_kernel.
__global__ __launch_bounds__(CNT) void chain_build_kernel(const double* __restrict__ d,
                                                          const double* __restrict__ alpha, int n,
                                                          const double* __restrict__ mu,
                                                          double* __restrict__ lv,
                                                          double* __restrict__ c,
                                                          ChainOut* out) {
  __shared__ double sh[CNT / 64 + 1];
  // member 0
  double s1 = 0.0, s2 = 0.0;
  for (int j = threadIdx.x; j < n; j += CNT) {
    const double a = alpha[j];
    lv[j] = a;
    s1 += a;
    s2 += a * d[j];
  }
  double S1_2 = block_sum<CNT>(s1, sh);
  double S2_2 = block_sum<CNT>(s2, sh);
  double c2 = 1.0;
  if (threadIdx.x == 0) c[0] = 1.0;
  if (n == 0) {
    if (threadIdx.x == 0) *out = ChainOut{1, 1};
    return;
  }
  // member 1 (p_0')
  double cs = 0.0;
  s1 = 0.0;
  s2 = 0.0;
  double* L1 = lv + level_off(n, 1);
  const double dl = d[n - 1];
  for (int j = threadIdx.x; j < n; j += CNT) {
    cs += mu[j];
    if (j < n - 1) {
      const double a = (dl - d[j]) * mu[j];
      L1[j] = a;
      s1 += a;
      s2 += a * d[j];
    }
  }
  double c1 = block_sum<CNT>(cs, sh);
  double S1_1 = block_sum<CNT>(s1, sh);
  double S2_1 = block_sum<CNT>(s2, sh);
  if (threadIdx.x == 0) c[1] = c1;
  if (!(c1 > 0.0)) {
    if (threadIdx.x == 0) *out = ChainOut{2, 0};
    return;
  }
  for (int m = 2; m <= n; ++m) {
    const double e1 = d[n - m], e2 = d[n - m + 1];
    const double A = c2 / c1;
    const double B = e2 + S1_2 / c2 - S1_1 / c1;
    const double cm = -(c2 * e1 * e2 + S1_2 * (e1 + e2) - S2_2) +
                      A * (c1 * B * e1 + S1_1 * (B + e1) - S2_1);
    const double* Lm2 = lv + level_off(n, m - 2);
    const double* Lm1 = lv + level_off(n, m - 1);
    double* Lm = lv + level_off(n, m);
    s1 = 0.0;
    s2 = 0.0;
    for (int j = threadIdx.x; j < n - m; j += CNT) {
      const double dj = d[j];
      const double a = -Lm2[j] * (dj - e1) * (dj - e2) + A * (dj - B) * Lm1[j] * (dj - e1);
      Lm[j] = a;
      s1 += a;
      s2 += a * dj;
    }
    if (threadIdx.x == 0) c[m] = cm;
    if (!(cm > 0.0)) {  // the same value in every thread: a uniform exit
      if (threadIdx.x == 0) *out = ChainOut{m + 1, 0};
      return;
    }
    const double S1_m = block_sum<CNT>(s1, sh);
    const double S2_m = block_sum<CNT>(s2, sh);
    c2 = c1;
    c1 = cm;
    S1_2 = S1_1;
    S2_2 = S2_1;
    S1_1 = S1_m;
    S2_1 = S2_m;
  }
  if (threadIdx.x == 0) *out = ChainOut{n + 1, 1};
}

__device__ __forceinline__ int count_below_sorted(const double* v, int n, double x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (v[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// counts[p] = eigenvalues of A' below x[p]: the chain's V(-inf) - V(x), plus the
// known zeros and the deflated eigenvalues below x; -1 when x is one of the
// chain's poles (the member signs are not defined there).  One block per point.
__global__ __launch_bounds__(256) void chain_count_kernel(
    const double* __restrict__ d, int n, const double* __restrict__ lv,
    const double* __restrict__ c, int levels, const double* __restrict__ xi, int n_xi,
    const double* __restrict__ dval, const DevInfo* info, const double* __restrict__ x,
    int64_t* __restrict__ counts) {
  __shared__ signed char s_sg[CHUNK];
  __shared__ int s_on_pole;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double xp = x[blockIdx.x];
  const int below = count_below_sorted(d, n, xp);
  if (threadIdx.x == 0) s_on_pole = (below < n && d[below] == xp) ? 1 : 0;
  __syncthreads();
  if (s_on_pole) {
    if (threadIdx.x == 0) counts[blockIdx.x] = -1;
    return;
  }
  int v_minus = 0, v_x = 0, last_minus = 0, last_x = 0;  // running changes (thread 0)
  for (int m0 = 0; m0 < levels; m0 += CHUNK) {
    const int mc = min(CHUNK, levels - m0);
    for (int q = wv; q < mc; q += 4) {
      const int m = m0 + q;
      const double* a = lv + level_off(n, m);
      double f = 0.0;
      for (int j = lane; j < n - m; j += 64) f += a[j] / (xp - d[j]);
      f = wave_sum(f);
      f = c[m] - f;
      const int above = max(0, (n - m) - below);
      int sg = (f > 0.0) - (f < 0.0);
      if (above & 1) sg = -sg;
      if (lane == 0) s_sg[q] = (signed char)sg;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int q = 0; q < mc; ++q) {
        const int m = m0 + q;
        const int sx = s_sg[q];
        if (sx != 0) {
          if (last_x != 0 && sx != last_x) ++v_x;
          last_x = sx;
        }
        int sm = (c[m] > 0.0) - (c[m] < 0.0);
        if ((n - m) & 1) sm = -sm;
        if (sm != 0) {
          if (last_minus != 0 && sm != last_minus) ++v_minus;
          last_minus = sm;
        }
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int known = count_below_sorted(xi, n_xi, xp);
    const int defl = count_below_sorted(dval, info->n_defl, xp);
    counts[blockIdx.x] = (int64_t)(v_minus - v_x) + known + defl;
  }
}

template <int K>
static hipError_t residue_launch(const Work& w, int n_d, double* alpha, hipStream_t s) {
  hipLaunchKernelGGL((residue_kernel<K>), dim3((n_d + 3) / 4), dim3(256), 0, s, w, alpha);
  return hipGetLastError();
}

hipError_t launch_chain(const Work& w, int n_d, const double* xi, int n_xi, double* ws,
                        int* bad, hipStream_t s) {
  // ws: alpha [n_d] | mu [n_d] | c [n_d + 1] | out (2 doubles) | levels (level_off(N, N+1))
  double* alpha = ws;
  double* mu = ws + n_d;
  double* c = mu + n_d;
  ChainOut* out = reinterpret_cast<ChainOut*>(c + n_d + 1);
  double* lv = c + n_d + 3;
  if (n_d > 0) {
    hipError_t e;
    switch (w.k) {
      case 1: e = residue_launch<1>(w, n_d, alpha, s); break;
      case 2: e = residue_launch<2>(w, n_d, alpha, s); break;
      case 3: e = residue_launch<3>(w, n_d, alpha, s); break;
      case 4: e = residue_launch<4>(w, n_d, alpha, s); break;
      case 5: e = residue_launch<5>(w, n_d, alpha, s); break;
      case 6: e = residue_launch<6>(w, n_d, alpha, s); break;
      case 7: e = residue_launch<7>(w, n_d, alpha, s); break;
      case 8: e = residue_launch<8>(w, n_d, alpha, s); break;
      default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
  }
  const int N = n_d - n_xi;
  if (n_xi > 0 && N > 0) {
    hipLaunchKernelGGL(chain_deflate_kernel, dim3((N + 255) / 256), dim3(256), 0, s, w.rd, n_d,
                       xi, n_xi, alpha, bad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const double* dch = w.rd + n_xi;
  const double* ach = alpha + n_xi;
  if (N > 0) {
    hipLaunchKernelGGL(chain_mu_kernel, dim3((N + 3) / 4), dim3(256), 0, s, dch, ach, N, mu);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(chain_build_kernel, dim3(1), dim3(CNT), 0, s, dch, ach, N, mu, lv, c, out);
  return hipGetLastError();
}

size_t chain_ws_doubles(int n_d) {
  return 3 * (size_t)n_d + 4 + level_off(n_d, n_d + 1);
}

hipError_t launch_chain_count(const Work& w, int n_d, const double* xi, int n_xi,
                              const double* ws, int levels, const double* x, int n_x,
                              int64_t* counts, hipStream_t s) {
  if (n_x <= 0) return hipSuccess;
  const double* c = ws + 2 * (size_t)n_d;
  const double* lv = c + n_d + 3;
  hipLaunchKernelGGL(chain_count_kernel, dim3(n_x), dim3(256), 0, s, w.rd + n_xi, n_d - n_xi, lv,
                     c, levels, xi, n_xi, w.dval, w.info, x, counts);
  return hipGetLastError();
}

}  // namespace eigupd
