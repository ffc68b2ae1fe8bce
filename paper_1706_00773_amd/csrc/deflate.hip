// deflate.hip -- bounds and deflation of the secular problem, one block.
//
// The secular function of eq. (1) needs distinct poles and nonzero rows of U
// (the rank-1 case of Sec. 1 states both conditions; eq. (4) assumes distinct
// poles).  This kernel prepares that reduced problem:
//   1. ahat = max|lambda| + ||U||_F^2 (a bound on ||A'||_2) and column norms
//      (for the outer Courant-Weyl bounds of Sec. 2.2);
//   2. rows with ||u_j|| ||U||_F <= TAU_ROW * ahat are dropped: (lambda_j, e_j)
//      is an eigenpair of the deflated problem;
//   3. runs of remaining rows whose poles are closer than TAU_GAP * ahat form a
//      group; a column-pivoted Householder QR of the group's m-by-k block of U
//      leaves r <= min(m, k) nonzero rows, which are kept as one multi-row pole
//      (value: the group's first pole); the other m - r rows are deflated;
//   4. compaction (block prefix sums) into the reduced arrays, segments and the
//      deflated list, all in ascending pole order.
// One block (1024 threads, 512 from k = 5); groups of two or more rows are rare and each is
// factorised by one thread.
#include "common.h"

namespace eigupd {

// Threads of the deflation block: 1024 up to k = 4, 512 from k = 5.  A 1024-thread
// block allows 128 VGPRs; from k = 3 the per-thread rows of U spill there
// (15 VGPRs at k = 3, 190 at k = 8).  Measured at n = 8192: 512 threads cost
// k = 4 24 us (99 -> 123 us; half the waves to hide latency) and saved k = 8
// 15 us (181 -> 166 us).
template <int K>
constexpr int dnt() { return (K <= 4) ? 1024 : 512; }

template <int K>
__device__ void group_qr(const Work& w, int g, double tol_abs, double* rem2) {
  const int first = w.g_first[g];
  const int m = w.g_m[g];
  double* R = w.urot + (size_t)first * K;
  for (int t = 0; t < m; ++t) {
    const int j = w.nt_list[first + t];
#pragma unroll
    for (int c = 0; c < K; ++c) R[(size_t)t * K + c] = w.U[(size_t)j * K + c];
  }
  unsigned used = 0;
  int r_eff = 0, nref = 0;
  for (int h = 0; h < m && h < K; ++h) {
    int best = -1;
    double bn = -1.0;
#pragma unroll
    for (int c = 0; c < K; ++c) {
      if ((used >> c) & 1u) continue;
      double s = 0.0;
      for (int t = h; t < m; ++t) s += R[(size_t)t * K + c] * R[(size_t)t * K + c];
      if (s > bn) {
        bn = s;
        best = c;
      }
    }
    if (best < 0 || sqrt(bn) <= tol_abs) break;
    r_eff = h + 1;
    if (h == m - 1) break;
    const double x0 = R[(size_t)h * K + best];
    const double alpha = -copysign(sqrt(bn), x0);
    const double vh = x0 - alpha;
    const double vtv = bn - x0 * x0 + vh * vh;
    const double beta = (vtv > 0.0) ? 2.0 / vtv : 0.0;
    double* hv = w.hv + (size_t)first * K;
    for (int t = h; t < m; ++t) hv[(size_t)t * K + h] = (t == h) ? vh : R[(size_t)t * K + best];
    w.hbeta[(size_t)g * K + h] = beta;
#pragma unroll
    for (int c = 0; c < K; ++c) {
      double d = 0.0;
      for (int t = h; t < m; ++t) d += hv[(size_t)t * K + h] * R[(size_t)t * K + c];
      d *= beta;
      for (int t = h; t < m; ++t) R[(size_t)t * K + c] -= d * hv[(size_t)t * K + h];
    }
    used |= 1u << best;
    nref = h + 1;
  }
  double rr = 0.0;
  for (int t = r_eff; t < m; ++t)
#pragma unroll
    for (int c = 0; c < K; ++c) rr += R[(size_t)t * K + c] * R[(size_t)t * K + c];
  *rem2 += rr;
  w.g_r[g] = r_eff;
  w.g_h[g] = nref;
}

template <int K>
__device__ __forceinline__ void deflate_body(const Work& w) {
  constexpr int DNT = dnt<K>();
  __shared__ double shd[DNT / 64 + 1];
  __shared__ int shi[DNT / 64 + 1];
  __shared__ int s_bad, s_odd;
  if (update_cancelled(w.st)) return;
  const int n = w.n, tid = threadIdx.x;
  const double* __restrict__ lam = w.lam_in;

  // 1. norms and bounds
  double cn[K];
#pragma unroll
  for (int c = 0; c < K; ++c) cn[c] = 0.0;
  double amax = 0.0;
  int bad = 0;
  for (int j = tid; j < n; j += DNT) {
    const double l = lam[j];
    amax = fmax(amax, fabs(l));
    bad |= !isfinite(l);
#pragma unroll
    for (int c = 0; c < K; ++c) {
      const double u = w.U[(size_t)j * K + c];
      cn[c] += u * u;
      bad |= !isfinite(u);
    }
  }
  if (tid == 0) s_bad = 0;
  __syncthreads();
  if (bad) atomicOr(&s_bad, 1);
  double colnorm[K];
  double fro = 0.0;
#pragma unroll
  for (int c = 0; c < K; ++c) {
    colnorm[c] = block_sum<DNT>(cn[c], shd);
    fro += colnorm[c];
  }
  amax = block_max<DNT>(amax, shd);
  __syncthreads();
  if (s_bad) {
    if (tid == 0) atomicOr(&w.st->status, ST_NONFINITE);
    return;
  }
  const double ahat = amax + fro;
  const double sfro = sqrt(fro);
  const double tol_abs = (sfro > 0.0) ? TAU_ROW * ahat / sfro : 0.0;  // on ||u_j||
  const double tol_gap = TAU_GAP * ahat;

  // The usual case: no tiny row and no two poles within tol_gap.  Every row is
  // then kept as a segment of its own and the reduced problem is the input: one
  // pass checks, one writes (the general phases below give the same arrays).
  if (tid == 0) s_odd = 0;
  __syncthreads();
  int odd = 0;
  for (int j = tid; j < n; j += DNT) {
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < K; ++c) s += w.U[(size_t)j * K + c] * w.U[(size_t)j * K + c];
    odd |= !(sqrt(s) > tol_abs);
    odd |= (j > 0) && !(lam[j] - lam[j - 1] > tol_gap);
  }
  if (odd) atomicOr(&s_odd, 1);
  __syncthreads();
  const bool plain = (s_odd == 0);
  double tiny2 = 0.0, spread = 0.0, rem2 = 0.0;
  int n_nt = n, n_mg = 0, ck = n, cd = 0, cs = n;
  for (int j = tid; plain && j < n; j += DNT) {
    w.rd[j] = lam[j];
#pragma unroll
    for (int c = 0; c < K; ++c) w.ru[(size_t)j * K + c] = w.U[(size_t)j * K + c];
    w.rrow[j] = j;
    w.row_seg[j] = j;
    w.seg_start[j] = j;
    w.seg_r[j] = 1;
    w.rmap[j] = j;
  }
  if (!plain) {
    // 2. tiny rows; compaction of the others (rmap temporarily holds the
    //    non-tiny position of each row, or -1)
    int carry = 0;
    for (int base = 0; base < n; base += DNT) {
      const int j = base + tid;
      int keep = 0;
      if (j < n) {
        double s = 0.0;
  #pragma unroll
        for (int c = 0; c < K; ++c) s += w.U[(size_t)j * K + c] * w.U[(size_t)j * K + c];
        const bool t = !(sqrt(s) > tol_abs);
        w.tiny[j] = t ? 1 : 0;
        keep = t ? 0 : 1;
        if (t) tiny2 += s;
      }
      int tot;
      const int ex = block_excl_scan<DNT>(keep, shi, &tot);
      if (j < n) {
        w.rmap[j] = keep ? carry + ex : -1;
        if (keep) w.nt_list[carry + ex] = j;
      }
      carry += tot;
    }
    n_nt = carry;
    __syncthreads();

    // 3. groups of near-equal poles among the non-tiny rows
    carry = 0;
    for (int base = 0; base < n_nt; base += DNT) {
      const int t = base + tid;
      int start = 0;
      if (t < n_nt) start = (t == 0) || (lam[w.nt_list[t]] - lam[w.nt_list[t - 1]] > tol_gap);
      int tot;
      const int ex = block_excl_scan<DNT>(start, shi, &tot);
      if (t < n_nt) {
        const int gid = carry + ex + start - 1;
        w.grp_id[t] = gid;
        if (start) w.g_first[gid] = t;
      }
      carry += tot;
    }
    const int n_groups = carry;
    __syncthreads();
    // Every group a single row (the usual case): no group records, reflectors or
    // QR are needed, and each kept row starts its own segment (phase 4's short
    // form below gives the same arrays as the general one).
    const bool singles = (n_groups == n_nt);
    carry = 0;
    for (int base = 0; !singles && base < n_groups; base += DNT) {
      const int g = base + tid;
      int multi = 0;
      if (g < n_groups) {
        const int f = w.g_first[g];
        const int next = (g + 1 < n_groups) ? w.g_first[g + 1] : n_nt;
        const int m = next - f;
        w.g_m[g] = m;
        w.g_val[g] = lam[w.nt_list[f]];
        w.g_r[g] = 1;
        w.g_h[g] = 0;
        multi = (m >= 2);
        if (multi) spread = fmax(spread, lam[w.nt_list[next - 1]] - lam[w.nt_list[f]]);
      }
      int tot;
      const int ex = block_excl_scan<DNT>(multi, shi, &tot);
      if (multi) w.mg_list[carry + ex] = g;
      carry += tot;
    }
    n_mg = carry;
    __syncthreads();
    for (int idx = tid; idx < n_mg; idx += DNT) group_qr<K>(w, w.mg_list[idx], tol_abs, &rem2);
    __syncthreads();

    // 4. reduced problem, segments and deflated list, in row order
    ck = 0;
    cd = 0;
    cs = 0;
    for (int base = 0; singles && base < n; base += DNT) {
      // rows kept exactly when not tiny; one scan gives the reduced row, the
      // segment (the same index) and, by difference, the deflated position
      const int j = base + tid;
      const int kept = (j < n && w.rmap[j] >= 0) ? 1 : 0;
      int tk;
      const int ek = block_excl_scan<DNT>(kept, shi, &tk);
      if (j < n) {
        if (kept) {
          const int ri = ck + ek;
          w.rd[ri] = lam[j];
  #pragma unroll
          for (int c = 0; c < K; ++c) w.ru[(size_t)ri * K + c] = w.U[(size_t)j * K + c];
          w.rrow[ri] = j;
          w.row_seg[ri] = cs + ek;
          w.seg_start[cs + ek] = ri;
          w.seg_r[cs + ek] = 1;
          w.rmap[j] = ri;
        } else {
          const int di = cd + tid - ek;
          w.dval[di] = lam[j];
          w.drow[di] = j;
          w.rmap[j] = -1;
        }
      }
      ck += tk;
      cs += tk;
      cd += min(DNT, n - base) - tk;
    }
    for (int base = 0; !singles && base < n; base += DNT) {
      const int j = base + tid;
      int kept = 0, defl = 0, segst = 0;
      int t = -1, g = -1, m = 1, pos = 0;
      if (j < n) {
        t = w.rmap[j];
        if (t < 0) {
          defl = 1;
        } else {
          g = w.grp_id[t];
          m = w.g_m[g];
          pos = t - w.g_first[g];
          kept = (m == 1) || (pos < w.g_r[g]);
          defl = !kept;
          segst = kept && (pos == 0);
        }
      }
      int tk, td, ts;
      const int ek = block_excl_scan<DNT>(kept, shi, &tk);
      const int ed = block_excl_scan<DNT>(defl, shi, &td);
      const int es = block_excl_scan<DNT>(segst, shi, &ts);
      if (kept) {
        const int ri = ck + ek;
        const int sid = cs + es + segst - 1;
        w.rd[ri] = (m == 1) ? lam[j] : w.g_val[g];
  #pragma unroll
        for (int c = 0; c < K; ++c)
          w.ru[(size_t)ri * K + c] = (m == 1) ? w.U[(size_t)j * K + c] : w.urot[(size_t)t * K + c];
        w.rrow[ri] = j;
        w.row_seg[ri] = sid;
        if (segst) {
          w.seg_start[sid] = ri;
          w.seg_r[sid] = (m == 1) ? 1 : w.g_r[g];
        }
      }
      if (defl) {
        const int di = cd + ed;
        w.dval[di] = lam[j];
        w.drow[di] = j;
      }
      if (j < n) w.rmap[j] = kept ? ck + ek : -1;
      ck += tk;
      cd += td;
      cs += ts;
    }
  }  // !plain
  const double t2 = block_sum<DNT>(tiny2 + rem2, shd);
  spread = block_max<DNT>(spread, shd);
  if (tid == 0) {
    const int n_d = ck;
    w.seg_start[cs] = n_d;
    DevInfo* info = w.info;
    info->n_d = n_d;
    info->n_s = cs;
    info->n_defl = cd;
    info->n_groups = n_mg;
    info->n_nt = n_nt;
    int p = 0;
#pragma unroll
    for (int c = 0; c < K; ++c) p += (w.sig_pos_mask >> c) & 1;
    info->p = p;
    info->q = K - p;
    info->k = K;
    info->ahat = ahat;
    info->fro2 = fro;
    double neg = 0.0, pos = 0.0;
#pragma unroll
    for (int c = 0; c < K; ++c) {
      if ((w.sig_pos_mask >> c) & 1)
        pos += colnorm[c];
      else
        neg += colnorm[c];
    }
    const double pad = 16.0 * 1.1102230246251565e-16 * ahat + 1e-300;
    if (n_d > 0) {
      info->lower = w.rd[0] - neg * (1.0 + 1e-10) - pad;
      info->upper = w.rd[n_d - 1] + pos * (1.0 + 1e-10) + pad;
    } else {
      info->lower = 0.0;
      info->upper = 0.0;
    }
    info->bwd = 2.0 * sqrt(t2) * sfro + t2 + spread;
    info->it_min = 0x7fffffff;
    info->it_max = 0;
    info->it_sum = 0;
    info->alpha_bad = 0;
    info->loc_alpha = 0;
    info->r_lo = 0;
    info->r_hi = n_d;
    info->e_lo = 0;
    info->e_hi = cd;
    info->root_next = 0;
  }
}

template <int K>
__global__ __launch_bounds__(dnt<K>()) void deflate_kernel(Work w) {
  deflate_body<K>(w);
}

// one block per instance
template <int K>
__global__ __launch_bounds__(dnt<K>()) void deflate_group(const Work* __restrict__ works) {
  deflate_body<K>(works[blockIdx.x]);
}

template <int K>
static hipError_t deflate_group_launch(const Work* works, int ninst, hipStream_t s) {
  hipLaunchKernelGGL((deflate_group<K>), dim3(ninst), dim3(dnt<K>()), 0, s, works);
  return hipGetLastError();
}

hipError_t launch_deflate_group(int k, const Work* works, int ninst, hipStream_t s) {
  if (ninst <= 0) return hipSuccess;
  EIGUPD_SWITCH_K(k, deflate_group_launch, works, ninst, s)
}

template <int K>
static hipError_t deflate_launch(const Work& w, hipStream_t s) {
  hipLaunchKernelGGL((deflate_kernel<K>), dim3(1), dim3(dnt<K>()), 0, s, w);
  return hipGetLastError();
}

hipError_t launch_deflate(const Work& w, hipStream_t s) {
  switch (w.k) {
    case 1: return deflate_launch<1>(w, s);
    case 2: return deflate_launch<2>(w, s);
    case 3: return deflate_launch<3>(w, s);
    case 4: return deflate_launch<4>(w, s);
    case 5: return deflate_launch<5>(w, s);
    case 6: return deflate_launch<6>(w, s);
    case 7: return deflate_launch<7>(w, s);
    case 8: return deflate_launch<8>(w, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace eigupd
