// smallmat.h -- k-by-k (k <= 8) symmetric linear algebra held in registers, one
// matrix per lane.  All loops have compile-time bounds and are unrolled, so the
// arrays stay in VGPRs.  Symmetric matrices are stored packed (upper triangle).
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
