// farfield.hip -- Q' = Q W (Sec. 2.4, eq. (10)) with the far blocks of W taken
// from Chebyshev expansions instead of being multiplied entry by entry.
//
// Every root column of W has the Cauchy-like form
//     W(j, p) = sum_a u_{j,a} c_{p,a} / (x_p - lambda_j)
// (x_p the point at which the column was formed, c_p its scaled null vector).
// Split the poles (rows) and the output columns, both in ascending order, into
// blocks of FF_B.  For a column block I and a row block J whose intervals are
// far apart (distance >= FF_ETA times the larger width), 1/(x - y) is smooth on
// both intervals and is replaced by its tensor Chebyshev interpolant of degree
// FF_P - 1 in each variable:
//     1/(x - y) ~ sum_{l,m} S_{I,l}(x) T_{IJ}(l, m) S_{J,m}(y),
//     T_{IJ}(l, m) = 1/(xhat_{I,l} - yhat_{J,m}),
// S the Lagrange basis of the first-kind Chebyshev nodes (barycentric form).
// The product then factors into three small products:
//     P2M  M_J = Q(:, J) B_J,          B_J(j, (m, a)) = u_{j,a} S_{J,m}(lambda_j)
//     M2L  L = M T                     (T zero on the near pairs)
//     L2P  Q'(:, I) += L_I Phi_I,      Phi_I((l, a), p) = S_{I,l}(x_p) c_{p,a}
// The near blocks are multiplied exactly: the band of row blocks I-1..I+1 around
// each column block, Q(:, band) W(band, I), plus up to FF_XR further pairs whose
// intervals are not far apart (a block widened by an outlying pole or root),
// Q(:, J) W(J, I).  Band, extra pairs and L2P are the segments of one product per
// column block, summed in registers and stored once.  A column block with more
// such pairs takes all rows as its band (no far field).  Deflated columns (unit
// vectors) lie in the band; deflated rows carry no charge.
//
// Layouts (column-major): M and L are (k n) x (nb P) with row (a, r) at a n + r,
// so that the columns (m, a) of one block form an n x kP matrix of leading
// dimension n; B is stored block by block (b_J x kP, leading dimension b_J);
// Phi is kP x n.
//
// The plan (intervals, near bands, descriptors) is made on the device, so the
// host does not wait.  When the update has merged equal-pole groups (W rows mixed
// by reflectors), a degenerate interval, half or more of the column blocks over
// all rows, or an error, the plan switches the product back to the dense kernel:
// of the two paths launched, each exits at once unless it was chosen.
#include "common.h"

namespace eigupd {

constexpr int FF_B = 256;        // rows / columns per block
constexpr int FF_P = 24;         // Chebyshev nodes per interval
// far: distance >= FF_ETA * max(width_I, width_J).  Along either interval the
// singularity of 1/(x - y) then lies outside the Bernstein ellipse of parameter
// rho = s + sqrt(s^2 - 1), s = 1 + 2 FF_ETA = 2 (rho = 2 + sqrt(3)), and the
// interpolant of FF_P = 24 nodes errs by at most about 1e-13 relative (7.5e-14
// measured at exactly that distance); pairs one width apart, which is what
// uniform spectra give, are at the rounding level (about 2e-15).  A factor of
// 0.7 (rho = 4.58, rounding level for every pair) cost 6% of the n = 8192
// update: the blocks at the ends of the spectrum, widened by the roots that the
// perturbation pushes outside it, gained extra near pairs.
constexpr double FF_ETA = 0.5;
constexpr int FF_MIN_N = 2048;   // below this the dense product is used
constexpr int FF_TILE = 128;     // tile side of the band / L2P products
constexpr int FF_PTILE = 64;     // tile side of the P2M products (N = kP is small)
constexpr int FF_MAXNB = 2048;   // blocks the plan handles (n up to 2^19)
constexpr int FF_XR = GSEG - 2;  // extra near pairs per column block

int ff_blocks(int n) { return n / FF_B; }
__host__ __device__ static inline int ff_bsize(int n, int nb, int i) {
  return i + 1 < nb ? FF_B : n - (nb - 1) * FF_B;
}
__host__ __device__ static inline int ff_tiles(int x) { return (x + FF_TILE - 1) / FF_TILE; }
__host__ __device__ static inline int ff_ptiles(int x) { return (x + FF_PTILE - 1) / FF_PTILE; }

bool ff_eligible(int n, int k) {
  return n >= FF_MIN_N && ff_blocks(n) <= FF_MAXNB && k >= 1 && k <= KMAX;
}

size_t ff_bytes(int n, int k) {
  const size_t nb = (size_t)ff_blocks(n), np = nb * FF_P, kp = (size_t)k * FF_P;
  size_t d = 2 * (size_t)k * n * np   // M, L
             + np * np                 // T
             + 2 * (size_t)n * kp      // B, Phi
             + 4 * nb + 2 * np;        // intervals, nodes
  size_t bytes = d * sizeof(double);
  bytes += nb * sizeof(GemmDescG) + nb * sizeof(GemmSegDesc) +
           (2 * (nb + 1) + 2 * nb + FF_XR * nb + 4) * sizeof(int);
  return bytes + 256;
}

FarField ff_layout(void* base, int n, int k) {
  FarField f;
  const size_t nb = (size_t)ff_blocks(n), np = nb * FF_P, kp = (size_t)k * FF_P;
  double* d = static_cast<double*>(base);
  f.n = n;
  f.k = k;
  f.nb = (int)nb;
  f.M = d;
  d += (size_t)k * n * np;
  f.L = d;
  d += (size_t)k * n * np;
  f.T = d;
  d += np * np;
  f.B = d;
  d += (size_t)n * kp;
  f.Phi = d;
  d += (size_t)n * kp;
  f.iv = d;
  d += 4 * nb;
  f.xn = d;
  d += np;
  f.yn = d;
  d += np;
  GemmDescG* g = reinterpret_cast<GemmDescG*>(d);
  f.desc = g;
  g += nb;
  GemmSegDesc* sg = reinterpret_cast<GemmSegDesc*>(g);
  f.seg = sg;
  sg += nb;
  int* ip = reinterpret_cast<int*>(sg);
  f.prefix = ip;
  ip += 2 * (nb + 1);
  f.near = ip;
  ip += 2 * nb;
  f.extra = ip;
  ip += FF_XR * nb;
  f.flags = ip;
  return f;
}

// Chebyshev node m of FF_P on [lo, hi] (c = ff_cos(m)) and its barycentric
// weight.
__device__ __forceinline__ double ff_cos(int m) { return cos((2 * m + 1) * M_PI / (2.0 * FF_P)); }
__device__ __forceinline__ double ff_node(double lo, double hi, double c) {
  return 0.5 * (lo + hi) + 0.5 * (hi - lo) * c;
}
__device__ __forceinline__ double ff_bw(int m) {
  const double s = sin((2 * m + 1) * M_PI / (2.0 * FF_P));
  return (m & 1) ? -s : s;
}

// Lagrange basis S_m(y), m < FF_P, of the nodes nd (second barycentric form;
// bw: the weights ff_bw).
__device__ __forceinline__ void ff_basis(const double* nd, const double* bw, double y,
                                         double* S) {
  int hit = -1;
  double sum = 0.0;
  for (int m = 0; m < FF_P; ++m) {
    const double dy = y - nd[m];
    if (dy == 0.0) hit = m;
    S[m] = bw[m] / (dy == 0.0 ? 1.0 : dy);
    sum += S[m];
  }
  if (hit >= 0) {
    for (int m = 0; m < FF_P; ++m) S[m] = (m == hit) ? 1.0 : 0.0;
  } else {
    const double r = 1.0 / sum;
    for (int m = 0; m < FF_P; ++m) S[m] *= r;
  }
}

// Absolute point at which column p was formed (deflated columns: its eigenvalue).
__device__ __forceinline__ double ff_colx(const Work& w, int p) {
  const ColParam& cp = w.colp[p];
  return cp.drow >= 0 ? w.lam_fin[p] : cp.d_o + cp.tau;
}

// One block per block index: the pole interval of row block J and the interval
// of the column points of column block J.
__global__ __launch_bounds__(256) void ff_interval_kernel(Work w, FarField f) {
  __shared__ double s_lo[4], s_hi[4];
  const int J = blockIdx.x, n = w.n, nb = f.nb;
  const int r0 = J * FF_B, b = ff_bsize(n, nb, J);
  double lo = INFINITY, hi = -INFINITY;
  for (int p = r0 + threadIdx.x; p < r0 + b; p += 256) {
    const double x = ff_colx(w, p);
    lo = fmin(lo, x);
    hi = fmax(hi, x);
  }
  lo = -wave_max(-lo);
  hi = wave_max(hi);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    s_lo[wv] = lo;
    s_hi[wv] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < 4; ++q) {
      s_lo[0] = fmin(s_lo[0], s_lo[q]);
      s_hi[0] = fmax(s_hi[0], s_hi[q]);
    }
    f.iv[4 * J + 0] = w.lam_in[r0];
    f.iv[4 * J + 1] = w.lam_in[r0 + b - 1];
    f.iv[4 * J + 2] = s_lo[0];
    f.iv[4 * J + 3] = s_hi[0];
  }
}

__device__ __forceinline__ bool ff_far(const double* iv, int I, int J) {
  const double ylo = iv[4 * J], yhi = iv[4 * J + 1], xlo = iv[4 * I + 2], xhi = iv[4 * I + 3];
  const double dist = fmax(xlo - yhi, ylo - xhi);
  return dist >= FF_ETA * fmax(xhi - xlo, yhi - ylo);
}

__device__ __forceinline__ GemmDescG ff_desc(const double* A, int lda, const double* B, int ldb,
                                             double* C, int ldc, int M, int N, int K, int bt) {
  GemmDescG g;
  g.A = A;
  g.B = B;
  g.C = C;
  g.M = M;
  g.N = N;
  g.K = K;
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.vec = !((lda & 1) || (ldb & 1) || (ldc & 1) || ((uintptr_t)A & 15) || ((uintptr_t)B & 15) ||
            ((uintptr_t)C & 15));
  g.tiles_m = (M + bt - 1) / bt;
  return g;
}

// One block: near bands and extra pairs, the path decision, nodes, descriptors
// and prefixes.
__global__ __launch_bounds__(256) void ff_plan_kernel(Work w, FarField f) {
  __shared__ int s_ok, s_full, s_cnt[FF_XR + 2];
  __shared__ unsigned char s_key[FF_MAXNB];  // segments beyond the band, per column block
  __shared__ short s_inv[FF_MAXNB];          // column block of each launch position
  __shared__ double s_c[FF_P];
  const int n = w.n, k = w.k, nb = f.nb, kp = k * FF_P;
  if (threadIdx.x == 0) {
    s_ok = (__builtin_nontemporal_load(&w.st->status) == 0) && (w.info->n_groups == 0);
    s_full = 0;
  }
  if (threadIdx.x < FF_XR + 2) s_cnt[threadIdx.x] = 0;
  if (threadIdx.x < FF_P) s_c[threadIdx.x] = ff_cos(threadIdx.x);
  __syncthreads();
  for (int I = threadIdx.x; I < nb; I += 256) {
    const double* iv = f.iv + 4 * I;
    const bool good = iv[1] > iv[0] && iv[3] > iv[2] && isfinite(iv[0]) && isfinite(iv[1]) &&
                      isfinite(iv[2]) && isfinite(iv[3]);
    if (!good) s_ok = 0;
  }
  __syncthreads();
  for (int I = threadIdx.x; I < nb; I += 256) {
    const int lo = max(0, I - 1), hi = min(nb - 1, I + 1);
    f.near[2 * I] = lo;
    f.near[2 * I + 1] = hi;
    int cnt = 0;
    if (s_ok)
      for (int J = 0; J < nb; ++J)
        if ((J < lo || J > hi) && !ff_far(f.iv, I, J)) {
          if (cnt < FF_XR) f.extra[I * FF_XR + cnt] = J;
          ++cnt;
        }
    int key = cnt;      // segments beyond the band (all rows: more than any)
    if (cnt > FF_XR) {  // this column block is multiplied exactly over all rows
      cnt = 0;
      key = FF_XR + 1;
      f.near[2 * I] = 0;
      f.near[2 * I + 1] = nb - 1;
      atomicAdd(&s_full, 1);
    }
    for (int r = cnt; r < FF_XR; ++r) f.extra[I * FF_XR + r] = -1;
    s_key[I] = (unsigned char)key;
    atomicAdd(&s_cnt[key], 1);
  }
  __syncthreads();
  // half or more of the column blocks over all rows: the dense product is cheaper
  if (threadIdx.x == 0 && 2 * s_full >= nb) s_ok = 0;
  __syncthreads();
  const bool ok = s_ok != 0;
  for (int e = threadIdx.x; e < nb * FF_P; e += 256) {
    const double* iv = f.iv + 4 * (e / FF_P);
    const double c = s_c[e % FF_P];
    f.yn[e] = ok ? ff_node(iv[0], iv[1], c) : 0.0;
    f.xn[e] = ok ? ff_node(iv[2], iv[3], c) : 0.0;
  }
  for (int I = threadIdx.x; I < nb; I += 256) {
    const int lo = f.near[2 * I], hi = f.near[2 * I + 1];
    const int b = ff_bsize(n, nb, I), r0 = I * FF_B;
    const int k0 = lo * FF_B, kn = (hi + 1 == nb ? n : (hi + 1) * FF_B) - k0;
    // P2M: M_I = Q(:, I) B_I
    f.desc[I] = ff_desc(w.Q_in + (size_t)r0 * n, n, f.B + (size_t)r0 * kp, b,
                        f.M + (size_t)I * FF_P * k * n, n, n, kp, b, FF_PTILE);
    // Q'(:, I) = Q(:, band) W(band, I) + sum_extra Q(:, J) W(J, I) + L_I Phi_I
    // Launch order of the column blocks' products: longer ones (more segments)
    // first, so that their tiles do not run last, alone, after the short ones
    // (stable in I; the tiles compute the same in any order).
    const int key = s_key[I];
    int pos = 0;
    for (int q = key + 1; q < FF_XR + 2; ++q) pos += s_cnt[q];
    for (int J = 0; J < I; ++J) pos += (s_key[J] == key) ? 1 : 0;
    s_inv[pos] = (short)I;
    GemmSegDesc& g = f.seg[pos];  // written in place
    int ns = 0, sl = 0;
    bool vec = !(n & 1) && !(kp & 1);
    auto add = [&](const double* A, const double* B, int ldb, int K) {
      g.A[ns] = A;
      g.B[ns] = B;
      g.lda[ns] = n;
      g.ldb[ns] = ldb;
      g.K[ns] = K;
      sl += (K + 15) / 16;
      g.send[ns] = sl;
      vec = vec && !((uintptr_t)A & 15) && !((uintptr_t)B & 15);
      ++ns;
    };
    add(w.Q_in + (size_t)k0 * n, w.W + (size_t)r0 * n + k0, n, kn);
    for (int r = 0; r < FF_XR; ++r) {
      const int J = ok ? f.extra[I * FF_XR + r] : -1;
      if (J >= 0) {
        const int j0 = J * FF_B;
        add(w.Q_in + (size_t)j0 * n, w.W + (size_t)r0 * n + j0, n, ff_bsize(n, nb, J));
      }
    }
    add(f.L + (size_t)I * FF_P * k * n, f.Phi + (size_t)r0 * kp, kp, kp);
    for (int r = ns; r < GSEG; ++r) {
      g.A[r] = g.B[r] = nullptr;
      g.lda[r] = g.ldb[r] = g.K[r] = 0;
      g.send[r] = sl;
    }
    g.C = w.Q_out + (size_t)r0 * n;
    g.M = n;
    g.N = b;
    g.ldc = n;
    g.vec = vec && !((uintptr_t)g.C & 15);
    g.tiles_m = ff_tiles(n);
    g.nseg = ns;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int tm = ff_tiles(n);
    int a = 0, c = 0;
    for (int I = 0; I < nb; ++I) {
      f.prefix[I] = c;
      f.prefix[(nb + 1) + I] = a;  // the I-th product launched
      a += tm * ff_tiles(ff_bsize(n, nb, s_inv[I]));
      c += ff_ptiles(n) * ff_ptiles(kp);
    }
    f.prefix[nb] = c;
    f.prefix[(nb + 1) + nb] = a;
    f.flags[0] = ok ? 0 : 1;                                             // far path skipped
    f.flags[1] = (ok || __builtin_nontemporal_load(&w.st->status) != 0) ? 1 : 0;  // dense skipped
  }
}

// T(( J, m), (I, l)) = 1/(xhat_{I,l} - yhat_{J,m}) on far pairs, 0 on near ones.
__global__ __launch_bounds__(256) void ff_t_kernel(FarField f) {
  if (__builtin_nontemporal_load(&f.flags[0]) != 0) return;
  const int np = f.nb * FF_P;
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long long)np * np) return;
  const int col = (int)(e / np), row = (int)(e % np);
  const int I = col / FF_P, J = row / FF_P;
  bool near = J >= f.near[2 * I] && J <= f.near[2 * I + 1];
  for (int r = 0; r < FF_XR; ++r) near = near || f.extra[I * FF_XR + r] == J;
  f.T[e] = near ? 0.0 : 1.0 / (f.xn[col] - f.yn[row]);
}

// Rows: B_J(j, m k + a) = u_{j,a} S_{J,m}(lambda_j).  Columns: Phi((l k + a), p) =
// S_{I,l}(x_p) c_{p,a} (zero for deflated columns).  Threads 0..n-1 take rows,
// n..2n-1 columns.
__global__ __launch_bounds__(256) void ff_weights_kernel(Work w, FarField f) {
  __shared__ double s_bw[FF_P];
  if (__builtin_nontemporal_load(&f.flags[0]) != 0) return;
  const int n = w.n, k = w.k, nb = f.nb, kp = k * FF_P;
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (threadIdx.x < FF_P) s_bw[threadIdx.x] = ff_bw(threadIdx.x);
  __syncthreads();
  if (t >= 2 * n) return;
  double S[FF_P];
  if (t < n) {
    const int r = t, J = min(r / FF_B, nb - 1), j = r - J * FF_B, b = ff_bsize(n, nb, J);
    const int jr = w.rmap[r];
    ff_basis(f.yn + J * FF_P, s_bw, w.lam_in[r], S);
    double* Bj = f.B + (size_t)J * FF_B * kp;
    for (int a = 0; a < k; ++a) {
      const double u = jr >= 0 ? w.ru[(size_t)jr * k + a] : 0.0;
      for (int m = 0; m < FF_P; ++m) Bj[(size_t)(m * k + a) * b + j] = u * S[m];
    }
  } else {
    const int p = t - n, I = min(p / FF_B, nb - 1);
    const ColParam& cp = w.colp[p];
    ff_basis(f.xn + I * FF_P, s_bw, ff_colx(w, p), S);
    double* ph = f.Phi + (size_t)p * kp;
    for (int a = 0; a < k; ++a) {
      const double c = cp.drow >= 0 ? 0.0 : cp.c[a];
      for (int l = 0; l < FF_P; ++l) ph[l * k + a] = S[l] * c;
    }
  }
}

hipError_t launch_ff_plan(const Work& w, const FarField& f, hipStream_t s) {
  if (f.nb < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(ff_interval_kernel, dim3(f.nb), dim3(256), 0, s, w, f);
  hipLaunchKernelGGL(ff_plan_kernel, dim3(1), dim3(256), 0, s, w, f);
  return hipGetLastError();
}

hipError_t launch_qw_farfield(const Work& w, const FarField& f, hipStream_t s) {
  const int n = w.n, k = w.k, nb = f.nb, kp = k * FF_P, np = nb * FF_P;
  if (nb < 1) return hipErrorInvalidValue;
  const long long ne = (long long)np * np;
  hipLaunchKernelGGL(ff_t_kernel, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, f);
  hipLaunchKernelGGL(ff_weights_kernel, dim3((2 * n + 255) / 256), dim3(256), 0, s, w, f);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int tm = ff_tiles(n);
  int band = 0;
  for (int I = 0; I < nb; ++I) band += tm * ff_tiles(ff_bsize(n, nb, I));
  const int p2m = nb * ff_ptiles(n) * ff_ptiles(kp);
  // the dense product, used when the plan rejected the far-field path
  e = launch_dgemm(n, n, n, w.Q_in, n, w.W, n, w.Q_out, n, f.flags + 1, s);
  if (e != hipSuccess) return e;
  e = launch_dgemm_desc(false, FF_PTILE, f.desc, f.prefix, nb, p2m, f.flags, s);
  if (e != hipSuccess) return e;
  e = launch_dgemm(k * n, np, np, f.M, k * n, f.T, np, f.L, k * n, f.flags, s);
  if (e != hipSuccess) return e;
  return launch_dgemm_seg(f.seg, f.prefix + (nb + 1), nb, band, f.flags, s);
}

}  // namespace eigupd
