// vectors.hip -- ordering of the new eigenvalues and the eigenvector matrix W
// in the Q basis (Sec. 2.4, eq. (10)).
//
// finalize   one block: absolute root values d_o + tau, made monotone by a
//            running maximum, merged with the deflated eigenvalues (ascending);
//            writes lambda' and one ColParam per output column.
// wbuild     W(j, p) = u_j^T c_p / (tau_p - (d_j - d_o,p)) for kept rows j of a
//            root column p (c_p is scaled so that the column has unit norm and
//            signed so that its entry at the first row of its origin pole is
//            positive); deflated columns are unit vectors.  Bound by the n^2
//            FP64 stores, which are coalesced (threads span rows).
// group_reflect  maps rows of W that belong to a merged equal-pole group back
//            from the rotated basis (Householder reflectors of the deflation).
// commit     counts the update as committed unless an error was raised.
#include "common.h"

namespace eigupd {

constexpr int FNT = 1024;

__device__ __forceinline__ int count_less(const double* v, int n, double x) {
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

__device__ __forceinline__ int count_less_equal(const double* v, int n, double x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (v[mid] <= x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Merges the roots [r_lo, r_hi) of the reduced problem (made monotone by a
// running maximum) with the deflated eigenvalues [e_lo, e_hi) (all of them for
// a full update) into lam_fin[0 ..) and one ColParam per output column.
// Running maximum of the absolute roots into xs (one block).
__device__ __forceinline__ void finalize_scan_body(const Work& w) {
  __shared__ double shd[FNT / 64];
  if (update_cancelled(w.st)) return;
  const int r_lo = w.info->r_lo, r_hi = w.info->r_hi;
  // absolute root values, running maximum: each thread takes one run of
  // consecutive roots, the runs' maxima are scanned across the block, then each
  // run is written.  Runs of up to FRUN roots are held in registers, their
  // loads issued together.
  constexpr int FRUN = 16;
  const int per = (r_hi - r_lo + FNT - 1) / FNT;
  const int b0 = min(r_hi, r_lo + (int)threadIdx.x * per), b1 = min(r_hi, b0 + per);
  auto xval = [&](int i) { return w.rd[w.seg_start[w.root_o[i]]] + w.root_tau[i]; };
  const bool in_regs = per <= FRUN;  // the same for every thread
  double x[FRUN];
  double run = -INFINITY;
  if (in_regs) {
#pragma unroll
    for (int e = 0; e < FRUN; ++e) x[e] = (b0 + e < b1) ? xval(b0 + e) : -INFINITY;
#pragma unroll
    for (int e = 0; e < FRUN; ++e) run = fmax(run, x[e]);
  } else {
    for (int i = b0; i < b1; ++i) run = fmax(run, xval(i));
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double v = wave_incl_max(run);
  if (lane == 63) shd[wv] = v;
  __syncthreads();
  double pre = __shfl_up(v, 1, 64);  // the maximum over the runs of lower lanes
  if (lane == 0) pre = -INFINITY;
  for (int q = 0; q < wv; ++q) pre = fmax(pre, shd[q]);
  if (in_regs) {
#pragma unroll
    for (int e = 0; e < FRUN; ++e) {
      pre = fmax(pre, x[e]);
      if (b0 + e < b1) w.xs[b0 + e] = pre;
    }
  } else {
    for (int i = b0; i < b1; ++i) {
      pre = fmax(pre, xval(i));
      w.xs[i] = pre;
    }
  }
}

// Output columns: merged eigenvalues and one ColParam each (threads t0, t0 +
// stride, ... of the roots and of the deflated eigenvalues); needs xs.
template <int K>
__device__ __forceinline__ void finalize_cols_body(const Work& w, int t0, int stride) {
  double* lam_dst = w.lam_fin;
  if (update_cancelled(w.st)) return;
  const int r_lo = w.info->r_lo, r_hi = w.info->r_hi;
  const int e_lo = w.info->e_lo, e_hi = w.info->e_hi;
  const double* dval = w.dval + e_lo;
  const int n_e = e_hi - e_lo, n_r = r_hi - r_lo;
  for (int i = r_lo + t0; i < r_hi; i += stride) {
    const double x = w.xs[i];
    const int pos = (i - r_lo) + count_less(dval, n_e, x);
    lam_dst[pos] = x;
    ColParam cp;
    const int o = w.root_o[i];
    const int jo = w.seg_start[o];
    cp.d_o = w.rd[jo];
    cp.tau = w.root_tv[i];
    double dot = 0.0;
#pragma unroll
    for (int c = 0; c < K; ++c) dot += w.ru[(size_t)jo * K + c] * w.root_c[(size_t)i * K + c];
    const double sgn = (dot / cp.tau < 0.0) ? -1.0 : 1.0;
#pragma unroll
    for (int c = 0; c < KMAX; ++c) cp.c[c] = (c < K) ? sgn * w.root_c[(size_t)i * K + c] : 0.0;
    cp.drow = -1;
    cp.pad = 0;
    w.colp[pos] = cp;
  }
  for (int j = t0; j < n_e; j += stride) {
    const double v = dval[j];
    const int pos = j + count_less_equal(w.xs + r_lo, n_r, v);
    lam_dst[pos] = v;
    ColParam cp;
    cp.d_o = 0.0;
    cp.tau = 0.0;
#pragma unroll
    for (int c = 0; c < KMAX; ++c) cp.c[c] = 0.0;
    cp.drow = w.drow[e_lo + j];
    cp.pad = 0;
    w.colp[pos] = cp;
  }
}

template <int K>
__device__ __forceinline__ void finalize_body(const Work& w) {
  finalize_scan_body(w);
  __syncthreads();
  finalize_cols_body<K>(w, threadIdx.x, FNT);
}

// W tile: 256 rows x CB columns per block (block coordinates bx, by).  The
// block's CB column parameters are read once into LDS (every thread needs all of
// them; read from global memory they were a chain of dependent scalar loads).
template <int K, int CB>
__device__ __forceinline__ void wbuild_body(const Work& w, int bx, int by) {
  static_assert(CB <= 256, "one thread per column parameter");
  __shared__ ColParam s_cp[CB];
  if (update_cancelled(w.st)) return;
  const int n = w.n;
  const int r = bx * 256 + threadIdx.x;
  const int p0 = by * CB;
  const int pe = min(w.ncols, p0 + CB);
  if ((int)threadIdx.x < pe - p0) s_cp[threadIdx.x] = w.colp[p0 + threadIdx.x];
  __syncthreads();
  if (r >= n) return;
  const int jr = w.rmap[r];
  double dj = 0.0, u[K];
#pragma unroll
  for (int c = 0; c < K; ++c) u[c] = 0.0;
  if (jr >= 0) {
    dj = w.rd[jr];
#pragma unroll
    for (int c = 0; c < K; ++c) u[c] = w.ru[(size_t)jr * K + c];
  }
  double* __restrict__ Wc = w.W;
  for (int p = p0; p < pe; ++p) {
    const ColParam& cp = s_cp[p - p0];
    double val;
    if (cp.drow >= 0) {
      val = (r == cp.drow) ? 1.0 : 0.0;
    } else {
      double num = 0.0;
#pragma unroll
      for (int c = 0; c < K; ++c) num = fma(u[c], cp.c[c], num);
      const double y = cp.tau - (dj - cp.d_o);
      val = (jr >= 0) ? num / y : 0.0;
    }
    Wc[(size_t)p * n + r] = val;
  }
}

// One wave per column; every merged group's rows are mapped back with
// H_0 H_1 ... H_{h-1} (the last reflector first).
template <int K>
__device__ __forceinline__ void group_reflect_body(const Work& w, int bid) {
  if (update_cancelled(w.st)) return;
  const int n_mg = w.info->n_groups;
  if (n_mg == 0) return;
  const int n = w.n;
  const int lane = threadIdx.x & 63;
  const int p = bid * 4 + (threadIdx.x >> 6);
  if (p >= w.ncols) return;
  double* col = w.W + (size_t)p * n;
  for (int gi = 0; gi < n_mg; ++gi) {
    const int g = w.mg_list[gi];
    const int first = w.g_first[g], m = w.g_m[g], h = w.g_h[g];
    for (int hh = h - 1; hh >= 0; --hh) {
      double d = 0.0;
      for (int t = hh + lane; t < m; t += 64)
        d += w.hv[(size_t)(first + t) * K + hh] * col[w.nt_list[first + t]];
      d = wave_sum(d) * w.hbeta[(size_t)g * K + hh];
      for (int t = hh + lane; t < m; t += 64)
        col[w.nt_list[first + t]] -= d * w.hv[(size_t)(first + t) * K + hh];
    }
  }
}

__device__ __forceinline__ void commit_body(const Work& w) {
  if (threadIdx.x == 0) {
    if (w.st->status == 0) w.st->gen += 1;
  }
}

constexpr int WB_CB = 32;  // W columns per wbuild block

template <int K>
__global__ __launch_bounds__(FNT) void finalize_kernel(Work w) {
  finalize_body<K>(w);
}
template <int K>
__global__ __launch_bounds__(FNT) void finalize_group(const Work* __restrict__ works) {
  finalize_body<K>(works[blockIdx.x]);
}
template <int K, int CB>
__global__ __launch_bounds__(256) void wbuild_kernel(Work w) {
  wbuild_body<K, CB>(w, blockIdx.x, blockIdx.y);
}
// Far-field product: only the rows of W it reads (the near band and the further
// near ranges of each column block, at the 256-row granularity of this kernel),
// all of W when its plan fell back to the dense product.
template <int K, int CB>
__global__ __launch_bounds__(256) void wbuild_ff_kernel(Work w, FarField f) {
  if (__builtin_nontemporal_load(&f.flags[0]) == 0) {
    const int I = min((int)blockIdx.y * CB / 256, f.nb - 1);
    const int t0 = blockIdx.x * 256, t1 = min(w.n, t0 + 256);  // rows of this tile
    auto hits = [&](int hlo, int hhi) {
      return hlo >= 0 && ff_row_begin(f, hlo) < t1 && ff_row_end(f, hhi) > t0;
    };
    bool need = hits(f.near[2 * I], f.near[2 * I + 1]);
    for (int r = 0; r < GSEG - 2; ++r)
      need = need || hits(f.extra[2 * (I * (GSEG - 2) + r)], f.extra[2 * (I * (GSEG - 2) + r) + 1]);
    if (!need) return;
  }
  wbuild_body<K, CB>(w, blockIdx.x, blockIdx.y);
}
template <int K, int CB>
__global__ __launch_bounds__(256) void wbuild_group(Group g) {
  const int i = group_instance(g, blockIdx.x);
  const Work& w = g.works[i];
  const int b = blockIdx.x - g.prefix[i];
  const int gx = (w.n + 255) / 256;
  wbuild_body<K, CB>(w, b % gx, b / gx);
}
template <int K>
__global__ __launch_bounds__(256) void group_reflect_kernel(Work w) {
  group_reflect_body<K>(w, blockIdx.x);
}
template <int K>
__global__ __launch_bounds__(256) void group_reflect_group(Group g) {
  const int i = group_instance(g, blockIdx.x);
  group_reflect_body<K>(g.works[i], blockIdx.x - g.prefix[i]);
}
__global__ void commit_kernel(Work w) { commit_body(w); }
__global__ void commit_group(const Work* __restrict__ works) { commit_body(works[blockIdx.x]); }

__global__ void zero_ints_kernel(int* p, int count) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
    p[i] = 0;
}

int wbuild_blocks(int n) { return ((n + 255) / 256) * ((n + WB_CB - 1) / WB_CB); }
int reflect_blocks(int n) { return (n + 3) / 4; }

__global__ __launch_bounds__(FNT) void finalize_scan_kernel(Work w) { finalize_scan_body(w); }
template <int K>
__global__ __launch_bounds__(256) void finalize_cols_kernel(Work w) {
  finalize_cols_body<K>(w, blockIdx.x * 256 + threadIdx.x, gridDim.x * 256);
}

// A single update: the scan in one block, the columns over the whole GPU (the
// same arithmetic as the one-block finalize of the grouped launches).
template <int K>
static hipError_t finalize_launch(const Work& w, hipStream_t s) {
  hipLaunchKernelGGL(finalize_scan_kernel, dim3(1), dim3(FNT), 0, s, w);
  hipLaunchKernelGGL((finalize_cols_kernel<K>), dim3((w.n + 255) / 256), dim3(256), 0, s, w);
  return hipGetLastError();
}

hipError_t launch_finalize(const Work& w, hipStream_t s) { EIGUPD_SWITCH_K(w.k, finalize_launch, w, s) }

template <int K>
static hipError_t wbuild_launch(const Work& w, hipStream_t s) {
  if (w.ncols <= 0) return hipSuccess;
  dim3 grid((w.n + 255) / 256, (w.ncols + WB_CB - 1) / WB_CB);
  hipLaunchKernelGGL((wbuild_kernel<K, WB_CB>), grid, dim3(256), 0, s, w);
  return hipGetLastError();
}

template <int K>
static hipError_t wbuild_ff_launch(const Work& w, const FarField& f, hipStream_t s) {
  static_assert(256 % WB_CB == 0, "column groups inside a far-field block");
  if (w.ncols <= 0) return hipSuccess;
  dim3 grid((w.n + 255) / 256, (w.ncols + WB_CB - 1) / WB_CB);
  hipLaunchKernelGGL((wbuild_ff_kernel<K, WB_CB>), grid, dim3(256), 0, s, w, f);
  return hipGetLastError();
}

hipError_t launch_wbuild_ff(const Work& w, const FarField& f, hipStream_t s) {
  EIGUPD_SWITCH_K(w.k, wbuild_ff_launch, w, f, s)
}

template <int K>
static hipError_t group_reflect_launch(const Work& w, hipStream_t s) {
  if (w.ncols <= 0) return hipSuccess;
  hipLaunchKernelGGL((group_reflect_kernel<K>), dim3((w.ncols + 3) / 4), dim3(256), 0, s, w);
  return hipGetLastError();
}

#define EIGUPD_DISPATCH_K2(fn)                \
  switch (w.k) {                              \
    case 1: return fn<1>(w, s);               \
    case 2: return fn<2>(w, s);               \
    case 3: return fn<3>(w, s);               \
    case 4: return fn<4>(w, s);               \
    case 5: return fn<5>(w, s);               \
    case 6: return fn<6>(w, s);               \
    case 7: return fn<7>(w, s);               \
    case 8: return fn<8>(w, s);               \
    default: return hipErrorInvalidValue;     \
  }

hipError_t launch_wbuild(const Work& w, hipStream_t s) { EIGUPD_DISPATCH_K2(wbuild_launch) }

hipError_t launch_group_reflect(const Work& w, hipStream_t s) {
  EIGUPD_DISPATCH_K2(group_reflect_launch)
}

hipError_t launch_commit(const Work& w, hipStream_t s) {
  hipLaunchKernelGGL(commit_kernel, dim3(1), dim3(64), 0, s, w);
  return hipGetLastError();
}

// ----- grouped launches (one rank k per launch; commit covers all instances)

template <int K>
static hipError_t finalize_group_launch(const Work* works, int ninst, hipStream_t s) {
  hipLaunchKernelGGL((finalize_group<K>), dim3(ninst), dim3(FNT), 0, s, works);
  return hipGetLastError();
}
template <int K>
static hipError_t wbuild_group_launch(const Group& g, int blocks, hipStream_t s) {
  hipLaunchKernelGGL((wbuild_group<K, WB_CB>), dim3(blocks), dim3(256), 0, s, g);
  return hipGetLastError();
}
template <int K>
static hipError_t reflect_group_launch(const Group& g, int blocks, hipStream_t s) {
  hipLaunchKernelGGL((group_reflect_group<K>), dim3(blocks), dim3(256), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_finalize_group(int k, const Work* works, int ninst, hipStream_t s) {
  if (ninst <= 0) return hipSuccess;
  EIGUPD_SWITCH_K(k, finalize_group_launch, works, ninst, s)
}
hipError_t launch_wbuild_group(int k, const Group& g, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  EIGUPD_SWITCH_K(k, wbuild_group_launch, g, blocks, s)
}
hipError_t launch_reflect_group(int k, const Group& g, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  EIGUPD_SWITCH_K(k, reflect_group_launch, g, blocks, s)
}
hipError_t launch_commit_group(const Work* works, int ninst, hipStream_t s) {
  if (ninst <= 0) return hipSuccess;
  hipLaunchKernelGGL(commit_group, dim3(ninst), dim3(64), 0, s, works);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// First-order perturbation estimate (Sec. 3, eq. (11) as read: the sum runs
// over v_i, denominators lambda_j - lambda_i, Sigma included):
//   lambda_j ~ lambda_j + u_j^T Sigma u_j,
//   W(i, j) = delta_ij + (u_i^T Sigma u_j) / (lambda_j - lambda_i)  (i != j, and
//             lambda_i != lambda_j),  V = Q W.
// 256 rows x 32 columns of W per block, like wbuild; the estimate keeps the
// original order of the eigenpairs.
// ---------------------------------------------------------------------------
template <int K, int CB>
__global__ __launch_bounds__(256) void perturb_w_kernel(Work w, double* lam_out) {
  if (update_cancelled(w.st)) return;
  const int n = w.n;
  const int r = blockIdx.x * 256 + threadIdx.x;
  const int p0 = blockIdx.y * CB;
  const int pe = min(n, p0 + CB);
  if (r >= n) return;
  double su[K];  // Sigma u_r
  double lr = w.lam_in[r];
#pragma unroll
  for (int c = 0; c < K; ++c)
    su[c] = (((w.sig_pos_mask >> c) & 1) ? 1.0 : -1.0) * w.U[(size_t)r * K + c];
  if (blockIdx.y == 0) {
    double d = 0.0;
#pragma unroll
    for (int c = 0; c < K; ++c) d = fma(su[c], w.U[(size_t)r * K + c], d);
    lam_out[r] = lr + d;
  }
  for (int p = p0; p < pe; ++p) {
    double val;
    const double lp = w.lam_in[p];
    if (p == r) {
      val = 1.0;
    } else if (lp == lr) {
      val = 0.0;
    } else {
      double num = 0.0;
#pragma unroll
      for (int c = 0; c < K; ++c) num = fma(su[c], w.U[(size_t)p * K + c], num);
      val = num / (lp - lr);
    }
    w.W[(size_t)p * n + r] = val;
  }
}

template <int K>
static hipError_t perturb_launch(const Work& w, double* lam_out, hipStream_t s) {
  dim3 grid((w.n + 255) / 256, (w.n + WB_CB - 1) / WB_CB);
  hipLaunchKernelGGL((perturb_w_kernel<K, WB_CB>), grid, dim3(256), 0, s, w, lam_out);
  return hipGetLastError();
}

hipError_t launch_perturb_w(const Work& w, double* lam_out, hipStream_t s) {
  EIGUPD_SWITCH_K(w.k, perturb_launch, w, lam_out, s)
}

}  // namespace eigupd
