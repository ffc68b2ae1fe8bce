// smallmat.h -- k-by-k (k <= 8) symmetric linear algebra held in registers.
// Either one matrix per lane (packed upper triangle; all loops have compile-time
// bounds and are unrolled, so the arrays stay in VGPRs), or, for the larger
// ranks, one matrix per group of 8 lanes with one row per lane.
#pragma once

#include <hip/hip_runtime.h>

namespace eigupd {

template <int N>
struct Sym {
  static constexpr int NS = N * (N + 1) / 2;
  // packed index of (r, c), r, c < N
  static __host__ __device__ constexpr int at(int r, int c) {
    return r <= c ? r * N - (r * (r - 1)) / 2 + (c - r) : c * N - (c * (c - 1)) / 2 + (r - c);
  }
};

// One plane rotation that annihilates a(p,q) (two-sided, symmetric Schur
// decomposition of the 2x2 block, Golub & Van Loan Sec. 8.5), applied to the
// packed matrix and, if VEC, to the columns of V.
// 1/x and 1/sqrt(x) from the hardware estimates refined by two Newton steps
// (to about one ulp): the rotation needs c^2 + s^2 = 1 to working precision,
// not correctly rounded quotients.
__device__ __forceinline__ double nr_recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ double nr_rsqrt(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  double e = fma(-hx * y, y, 0.5);
  y = fma(y, e, y);
  e = fma(-hx * y, y, 0.5);
  return fma(y, e, y);
}

template <int N, int P, int Qc, bool VEC>
__device__ __forceinline__ void jacobi_rotate(double (&a)[Sym<N>::NS], double (&V)[N][N]) {
  constexpr int ipq = Sym<N>::at(P, Qc), ipp = Sym<N>::at(P, P), iqq = Sym<N>::at(Qc, Qc);
  const double apq = a[ipq];
  const bool z = (apq == 0.0);
  const double theta = z ? 0.0 : (a[iqq] - a[ipp]) * nr_recip(2.0 * apq);
  const double at = fabs(theta);
  // t = sign(theta) / (|theta| + sqrt(theta^2 + 1)); for huge theta, 1 / (2 theta)
  const double h = fma(theta, theta, 1.0);
  double t = (at > 1e150) ? 0.5 * nr_recip(theta)
                          : copysign(1.0, theta) * nr_recip(at + h * nr_rsqrt(h));
  t = (z || !(at == at)) ? 0.0 : t;
  const double c = nr_rsqrt(fma(t, t, 1.0));
  const double s = t * c;
  a[ipp] -= t * apq;
  a[iqq] += t * apq;
  a[ipq] = 0.0;
#pragma unroll
  for (int r = 0; r < N; ++r) {
    if (r == P || r == Qc) continue;
    const double g = a[Sym<N>::at(r, P)], h = a[Sym<N>::at(r, Qc)];
    a[Sym<N>::at(r, P)] = c * g - s * h;
    a[Sym<N>::at(r, Qc)] = s * g + c * h;
  }
  if (VEC) {
#pragma unroll
    for (int r = 0; r < N; ++r) {
      const double g = V[r][P], h = V[r][Qc];
      V[r][P] = c * g - s * h;
      V[r][Qc] = s * g + c * h;
    }
  }
}

template <int N, int P, int Qc, bool VEC>
struct SweepRow {
  static __device__ __forceinline__ void run(double (&a)[Sym<N>::NS], double (&V)[N][N]) {
    jacobi_rotate<N, P, Qc, VEC>(a, V);
    SweepRow<N, P, Qc + 1, VEC>::run(a, V);
  }
};
template <int N, int P, bool VEC>
struct SweepRow<N, P, N, VEC> {
  static __device__ __forceinline__ void run(double (&)[Sym<N>::NS], double (&)[N][N]) {}
};
template <int N, int P, bool VEC>
struct Sweep {
  static __device__ __forceinline__ void run(double (&a)[Sym<N>::NS], double (&V)[N][N]) {
    SweepRow<N, P, P + 1, VEC>::run(a, V);
    Sweep<N, P + 1, VEC>::run(a, V);
  }
};
template <int N, bool VEC>
struct Sweep<N, N, VEC> {
  static __device__ __forceinline__ void run(double (&)[Sym<N>::NS], double (&)[N][N]) {}
};

// Cyclic Jacobi: on return a is diagonal to working precision; its diagonal
// holds the eigenvalues and (VEC) column m of V the unit eigenvector of a(m,m).
template <int N, bool VEC>
__device__ inline void jacobi_eig(double (&a)[Sym<N>::NS], double (&V)[N][N]) {
  if (VEC) {
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int c = 0; c < N; ++c) V[r][c] = (r == c) ? 1.0 : 0.0;
  }
  if (N == 1) return;
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, dg = 0.0;
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int c = r; c < N; ++c) {
        const double v = a[Sym<N>::at(r, c)] * a[Sym<N>::at(r, c)];
        if (r == c)
          dg += v;
        else
          off += v;
      }
    if (!(off > 1e-36 * (dg + off))) break;
    Sweep<N, 0, VEC>::run(a, V);
  }
}

// The cyclic Jacobi of jacobi_eig without V: instead every rotation is also
// applied to a second packed symmetric matrix b, b <- J^T b J.  On return a is
// diagonal (the eigenvalues of a) and b = V^T b V in the eigenvector basis, so
// that for instance tr(a^{-1} b) = sum_m b(m,m) / a(m,m) needs no V.
template <int N, int P, int Qc>
__device__ __forceinline__ void jacobi_rotate_pair(double (&a)[Sym<N>::NS],
                                                   double (&b)[Sym<N>::NS]) {
  constexpr int ipq = Sym<N>::at(P, Qc), ipp = Sym<N>::at(P, P), iqq = Sym<N>::at(Qc, Qc);
  const double apq = a[ipq];
  const bool z = (apq == 0.0);
  const double theta = z ? 0.0 : (a[iqq] - a[ipp]) * nr_recip(2.0 * apq);
  const double at = fabs(theta);
  const double h = fma(theta, theta, 1.0);
  double t = (at > 1e150) ? 0.5 * nr_recip(theta)
                          : copysign(1.0, theta) * nr_recip(at + h * nr_rsqrt(h));
  t = (z || !(at == at)) ? 0.0 : t;
  const double c = nr_rsqrt(fma(t, t, 1.0));
  const double s = t * c;
  a[ipp] -= t * apq;
  a[iqq] += t * apq;
  a[ipq] = 0.0;
  {
    // the 2 x 2 block of b: [c -s; s c] [bpp bpq; bpq bqq] [c s; -s c]
    const double bpp = b[ipp], bqq = b[iqq], bpq = b[ipq];
    const double x = c * bpp - s * bpq, y = c * bpq - s * bqq;  // row p of J^T b
    const double x2 = s * bpp + c * bpq, y2 = s * bpq + c * bqq;  // row q of J^T b
    b[ipp] = x * c - y * s;
    b[ipq] = x * s + y * c;
    b[iqq] = x2 * s + y2 * c;
  }
#pragma unroll
  for (int r = 0; r < N; ++r) {
    if (r == P || r == Qc) continue;
    const double g = a[Sym<N>::at(r, P)], h2 = a[Sym<N>::at(r, Qc)];
    a[Sym<N>::at(r, P)] = c * g - s * h2;
    a[Sym<N>::at(r, Qc)] = s * g + c * h2;
    const double gb = b[Sym<N>::at(r, P)], hb = b[Sym<N>::at(r, Qc)];
    b[Sym<N>::at(r, P)] = c * gb - s * hb;
    b[Sym<N>::at(r, Qc)] = s * gb + c * hb;
  }
}

template <int N, int P, int Qc>
struct PairRow {
  static __device__ __forceinline__ void run(double (&a)[Sym<N>::NS], double (&b)[Sym<N>::NS]) {
    jacobi_rotate_pair<N, P, Qc>(a, b);
    PairRow<N, P, Qc + 1>::run(a, b);
  }
};
template <int N, int P>
struct PairRow<N, P, N> {
  static __device__ __forceinline__ void run(double (&)[Sym<N>::NS], double (&)[Sym<N>::NS]) {}
};
template <int N, int P>
struct PairSweep {
  static __device__ __forceinline__ void run(double (&a)[Sym<N>::NS], double (&b)[Sym<N>::NS]) {
    PairRow<N, P, P + 1>::run(a, b);
    PairSweep<N, P + 1>::run(a, b);
  }
};
template <int N>
struct PairSweep<N, N> {
  static __device__ __forceinline__ void run(double (&)[Sym<N>::NS], double (&)[Sym<N>::NS]) {}
};

template <int N>
__device__ inline void jacobi_eig_congruent(double (&a)[Sym<N>::NS], double (&b)[Sym<N>::NS]) {
  if (N == 1) return;
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, dg = 0.0;
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int c = r; c < N; ++c) {
        const double v = a[Sym<N>::at(r, c)] * a[Sym<N>::at(r, c)];
        if (r == c)
          dg += v;
        else
          off += v;
      }
    if (!(off > 1e-36 * (dg + off))) break;
    PairSweep<N, 0>::run(a, b);
  }
}

// ---------------------------------------------------------------------------
// The same eigensolve on an aligned group of 8 lanes: lane l of the group holds
// row l of the N x N symmetric matrix (a) and row l of V (v); lanes l >= N hold
// zero rows.  Cyclic Jacobi in the parallel ordering (the round-robin ordering of
// Golub & Van Loan Sec. 8.5.5): one sweep is NE - 1 steps (NE = N rounded up to
// even), each rotating NE / 2 disjoint pairs (p, q) at once, A <- J^T A J and
// V <- V J, with each pair's rotation chosen from (a_pp, a_qq, a_pq) as in
// jacobi_rotate.  A lane keeps only two rows in registers, where one matrix per
// lane needs all of A and V.
//
// Every lane of the wave calls it (the groups exchange rows by shuffles).  A
// group that is not `live`, or whose matrix has converged, applies identity
// rotations, which leave its rows bitwise unchanged: its result does not depend
// on the other groups of the wave.
// ---------------------------------------------------------------------------

// Partner of player j in step s of the round-robin ordering of NE (even)
// players (the circle method): over the NE - 1 steps every pair meets once.
template <int NE>
__host__ __device__ constexpr int rr_partner(int j, int s) {
  return (j == NE - 1) ? s : (j == s) ? NE - 1 : (2 * s - j + 2 * (NE - 1)) % (NE - 1);
}

__device__ __forceinline__ double group8_sum(double x) {
  x += __shfl_xor(x, 1, 64);
  x += __shfl_xor(x, 2, 64);
  return x + __shfl_xor(x, 4, 64);
}
__device__ __forceinline__ double group8_min(double x) {
  x = fmin(x, __shfl_xor(x, 1, 64));
  x = fmin(x, __shfl_xor(x, 2, 64));
  return fmin(x, __shfl_xor(x, 4, 64));
}
__device__ __forceinline__ int group8_sum_int(int x) {
  x += __shfl_xor(x, 1, 64);
  x += __shfl_xor(x, 2, 64);
  return x + __shfl_xor(x, 4, 64);
}

// Element j of a row held in registers, j a lane-dependent index.
template <int N>
__device__ __forceinline__ double row_at(const double (&a)[N], int j) {
  double x = 0.0;
#pragma unroll
  for (int c = 0; c < N; ++c) x = (c == j) ? a[c] : x;
  return x;
}

template <int N, bool VEC>
__device__ inline void jacobi_eig_rows(double (&a)[N], double (&v)[N], bool live) {
  constexpr int NE = N + (N & 1);
  const int lane = threadIdx.x & 63;
  const int l = lane & 7, base = lane & ~7;
  if (VEC) {
#pragma unroll
    for (int c = 0; c < N; ++c) v[c] = (c == l) ? 1.0 : 0.0;
  }
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, dg = 0.0;
#pragma unroll
    for (int c = 0; c < N; ++c) {
      const double x = a[c] * a[c];
      if (c == l)
        dg += x;
      else
        off += x;
    }
    // both triangles were summed
    off = 0.5 * group8_sum(off);
    dg = group8_sum(dg);
    const bool rot = live && (off > 1e-36 * (dg + off));
    if (__ballot(rot) == 0ull) break;
#pragma unroll
    for (int st = 0; st < NE - 1; ++st) {
      const int pr = (l < N) ? rr_partner<NE>(l, st) : l;
      const int pi = (pr < N) ? pr : l;  // no partner: the lane's row stays
      const double dl = row_at<N>(a, l), alp = row_at<N>(a, pi);
      const double dp = __shfl(dl, base + pi, 64);
      // the rotation of the pair (l, pi), from its lower lane
      double t = 0.0;
      if (rot && l < pi && alp != 0.0) {
        const double theta = (dp - dl) * nr_recip(2.0 * alp);
        const double at = fabs(theta);
        const double h = fma(theta, theta, 1.0);
        t = (at > 1e150) ? 0.5 * nr_recip(theta)
                         : copysign(1.0, theta) * nr_recip(at + h * nr_rsqrt(h));
        t = (at == at) ? t : 0.0;
      }
      // an identity rotation exactly where there is none (c = 1, s = 0)
      const double c = (t == 0.0) ? 1.0 : nr_rsqrt(fma(t, t, 1.0));
      const double sn = t * c;
      // every pair's rotation, from its lower lane
      double cp[N], sp[N];
#pragma unroll
      for (int p = 0; p < N; ++p) {
        const int q = rr_partner<NE>(p, st);
        cp[p] = 1.0;
        sp[p] = 0.0;
        if (q < N && p < q) {
          cp[p] = __shfl(c, base + p, 64);
          sp[p] = __shfl(sn, base + p, 64);
        }
      }
      // A J and V J on this lane's rows; the own pair's rotation
      double co = 1.0, so = 0.0;
#pragma unroll
      for (int p = 0; p < N; ++p) {
        const int q = rr_partner<NE>(p, st);
        if (q < N && p < q) {
          {
            const double g = a[p], h2 = a[q];
            a[p] = cp[p] * g - sp[p] * h2;
            a[q] = sp[p] * g + cp[p] * h2;
          }
          if (VEC) {
            const double g = v[p], h2 = v[q];
            v[p] = cp[p] * g - sp[p] * h2;
            v[q] = sp[p] * g + cp[p] * h2;
          }
          if (l == p || l == q) {
            co = cp[p];
            so = sp[p];
          }
        }
      }
      // J^T (A J): rows l and pi combine
      double o[N];
#pragma unroll
      for (int c2 = 0; c2 < N; ++c2) o[c2] = __shfl(a[c2], base + pi, 64);
      if (l < pi) {
#pragma unroll
        for (int c2 = 0; c2 < N; ++c2) a[c2] = co * a[c2] - so * o[c2];
      } else if (l > pi) {
#pragma unroll
        for (int c2 = 0; c2 < N; ++c2) a[c2] = so * o[c2] + co * a[c2];
      }
      // the annihilated entry
      if (rot && pi != l) {
#pragma unroll
        for (int c2 = 0; c2 < N; ++c2) a[c2] = (c2 == pi) ? 0.0 : a[c2];
      }
    }
  }
}

// Number of negative eigenvalues of the packed symmetric matrix a (destroyed).
template <int N>
__device__ inline int neg_count(double (&a)[Sym<N>::NS]) {
  double V[N][N];
  jacobi_eig<N, false>(a, V);
  int neg = 0;
#pragma unroll
  for (int m = 0; m < N; ++m) neg += (a[Sym<N>::at(m, m)] < 0.0) ? 1 : 0;
  return neg;
}

// x^T B y for packed symmetric B.
template <int N>
__device__ __forceinline__ double quad(const double (&B)[Sym<N>::NS], const double* x,
                                       const double* y) {
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int b = 0; b < N; ++b) s += x[a] * B[Sym<N>::at(a, b)] * y[b];
  return s;
}

// Inertia of T restricted to the orthogonal complement of the row space of the
// r-by-N matrix Y (rows 0..r-1 of Yrows, full row rank, 0 <= r <= N): returns
// the number of negative eigenvalues of P^T T P, P an orthonormal basis of that
// complement.  Householder reflectors H_h (zeroing Y^T below row h) are applied
// to T as similarities; the leading r coordinates are then masked off.
template <int N>
__device__ inline int neg_count_compressed(double (&T)[Sym<N>::NS], double (&Y)[N][N], int r) {
#pragma unroll
  for (int h = 0; h < N; ++h) {
    if (h < r) {
      double nrm2 = 0.0;
#pragma unroll
      for (int i = h; i < N; ++i) nrm2 += Y[h][i] * Y[h][i];
      const double alpha = -copysign(sqrt(nrm2), Y[h][h]);
      double v[N];
#pragma unroll
      for (int i = 0; i < N; ++i) v[i] = (i < h) ? 0.0 : Y[h][i];
      v[h] -= alpha;
      double vtv = 0.0;
#pragma unroll
      for (int i = h; i < N; ++i) vtv += v[i] * v[i];
      const double beta = (vtv > 0.0) ? 2.0 / vtv : 0.0;
      // remaining rows of Y
#pragma unroll
      for (int g = h + 1; g < N; ++g) {
        if (g < r) {
          double d = 0.0;
#pragma unroll
          for (int i = h; i < N; ++i) d += v[i] * Y[g][i];
          d *= beta;
#pragma unroll
          for (int i = h; i < N; ++i) Y[g][i] -= d * v[i];
        }
      }
      // T <- H T H with H = I - beta v v^T
      double p[N];
#pragma unroll
      for (int a = 0; a < N; ++a) {
        double s = 0.0;
#pragma unroll
        for (int b = h; b < N; ++b) s += T[Sym<N>::at(a, b)] * v[b];
        p[a] = beta * s;
      }
      double kk = 0.0;
#pragma unroll
      for (int a = h; a < N; ++a) kk += v[a] * p[a];
      kk *= 0.5 * beta;
      double w[N];
#pragma unroll
      for (int a = 0; a < N; ++a) w[a] = p[a] - kk * v[a];
#pragma unroll
      for (int a = 0; a < N; ++a)
#pragma unroll
        for (int b = a; b < N; ++b) T[Sym<N>::at(a, b)] -= v[a] * w[b] + w[a] * v[b];
    }
  }
#pragma unroll
  for (int a = 0; a < N; ++a)
#pragma unroll
    for (int b = a; b < N; ++b)
      if (a < r || b < r) T[Sym<N>::at(a, b)] = (a == b) ? 1.0 : 0.0;
  return neg_count<N>(T);
}

}  // namespace eigupd
