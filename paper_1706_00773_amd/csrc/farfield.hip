// farfield.hip -- Q' = Q W (Sec. 2.4, eq. (10)) with the far blocks of W taken
// from Chebyshev expansions instead of being multiplied entry by entry.
//
// Every root column of W has the Cauchy-like form
//     W(j, p) = sum_a u_{j,a} c_{p,a} / (x_p - lambda_j)
// (x_p the point at which the column was formed, c_p its scaled null vector).
// The output columns, in ascending order, are split into column blocks of FF_B;
// the poles (rows), also ascending, into row blocks of rb rows (FF_B for ranks
// above 2, FF_B / 2 up to rank 2).  For a column block I and a row block h whose
// intervals are far apart (distance >= etac times the column width and >= etar
// times the row width), 1/(x - y) is smooth on both intervals and is replaced by
// its tensor Chebyshev interpolant of pc nodes in x and pr nodes in y:
//     1/(x - y) ~ sum_{l,m} S_{I,l}(x) T_{Ih}(l, m) S_{h,m}(y),
//     T_{Ih}(l, m) = 1/(xhat_{I,l} - yhat_{h,m}),
// S the Lagrange basis of the first-kind Chebyshev nodes (barycentric form).
// The product then factors into three small products:
//     P2M  M_h = Q(:, h) B_h,          B_h(j, (m, a)) = u_{j,a} S_{h,m}(lambda_j)
//     M2L  L = M T                     (T zero on the near pairs)
//     L2P  Q'(:, I) += L_I Phi_I,      Phi_I((l, a), p) = S_{I,l}(x_p) c_{p,a}
// The near rows are multiplied exactly: the band of rows within rb of column
// block I (widened while the next row block is not far), Q(:, band) W(band, I),
// plus up to FF_XR further ranges of row blocks that are not far (blocks widened
// by outlying poles or roots), Q(:, R) W(R, I).  Band, further ranges and L2P are
// the segments of one product per column block, summed in registers and stored
// once.  A column block with more ranges takes all rows as its band (no far
// field).  Deflated columns (unit vectors) lie in the band; deflated rows carry
// no charge.
//
// Why half-width row blocks up to rank 2: the exact band shrinks from 3 FF_B to
// 2 FF_B rows (the band is 80% of the flops at FF_B rows), while M2L grows as
// k n (nr pr)(nb pc); from rank 3 the larger M2L costs what the band saves.
//
// Layouts (column-major): M is (k n) x (nr pr) and L (k n) x (nb pc), row (a, r)
// at a n + r, so that the columns (m, a) of one block form an n x k pr (or k pc)
// matrix of leading dimension n; B is stored block by block (b_h x k pr, leading
// dimension b_h); Phi is k pc x n.
//
// The plan (intervals, near rows, descriptors) is made on the device, so the
// host does not wait.  When the update has merged equal-pole groups (W rows mixed
// by reflectors), a degenerate interval, half or more of the column blocks with
// half the rows or more exact, or an error, the plan switches the product back
// to the dense kernel: of the two paths launched, each exits at once unless it
// was chosen.
#include "common.h"

namespace eigupd {

constexpr int FF_B = 256;        // columns per column block
constexpr int FF_PMAX = 32;      // most nodes per interval
constexpr int FF_MIN_N = 2048;   // below this the dense product is used
constexpr int FF_TILE = 128;     // tile side of the band / L2P products
constexpr int FF_PTILE = 64;     // tile side of the P2M products (N = k pr is small)
constexpr int FF_MAXNB = 2048;   // column blocks the plan handles (n up to 2^19)
constexpr int FF_XR = GSEG - 2;  // further near ranges per column block

// Row block size, nodes and separation factors by rank.  Interpolating
// 1/(x - y) in x over a column interval of width w, with the singularity at
// distance d, errs by about 4 rho^(-pc), rho = s + sqrt(s^2 - 1), s = 1 + 2 d / w
// (the factor 4 measured); the same holds in y with pr and the row width.
//  - Ranks above 2: rb = FF_B, pr = pc = 20, far when d >= 0.78 of both widths:
//    rho = 4.92 at the limit, about 6e-14; blocks one width apart, which is what
//    uniform spectra give, are at the rounding level.  24 nodes with a factor of
//    0.5 (7.5e-14 at its limit) made M2L 44% larger: n = 8192 updates at rank 4
//    and 8 ran at 232 and 127 updates/s against 243 and 134.
//  - Up to rank 2: rb = FF_B / 2.  The row blocks next to the band lie about
//    half a column width away (one row block between).  Columns: etac = 0.45,
//    pc = 24 (rho = 3.52, about 3e-13 relative at the limit, 7.5e-14 at half a
//    width); rows: etar = 0.85, pr = 20 (rho = 5.21, about 2e-14 at the limit;
//    those row blocks are one row width away).  With uniform spectra about one
//    in four of those row blocks falls inside a limit (random spacing) and is
//    multiplied exactly.  pr = 22 with etar = 0.675 (the same error at its
//    limit, fewer such blocks) took 0.025 ms more per n = 8192 update.  pc = 32 with etac = 0.35 (1e-15 at the limit) was
//    measured at n = 8192: M2L's 1024 column tiles instead of 768 took 0.15 ms
//    more per update, with the same residual and orthogonality against eigh.
struct FfCfg {
  int rb, pr, pc;
  double etar, etac;
};
__host__ __device__ static inline FfCfg ff_cfg(int k) {
  return k <= 2 ? FfCfg{FF_B / 2, 20, 24, 0.85, 0.45} : FfCfg{FF_B, 20, 20, 0.78, 0.78};
}

int ff_blocks(int n) { return n / FF_B; }
__host__ __device__ static inline int ff_bsize(int n, int nb, int i, int bs) {
  return i + 1 < nb ? bs : n - (nb - 1) * bs;
}
__host__ __device__ static inline int ff_tiles(int x) { return (x + FF_TILE - 1) / FF_TILE; }
__host__ __device__ static inline int ff_ptiles(int x) { return (x + FF_PTILE - 1) / FF_PTILE; }

bool ff_eligible(int n, int k) {
  return n >= FF_MIN_N && ff_blocks(n) <= FF_MAXNB && k >= 1 && k <= KMAX;
}

size_t ff_bytes(int n, int k) {
  const FfCfg c = ff_cfg(k);
  const size_t nb = (size_t)ff_blocks(n), nr = (size_t)(n / c.rb);
  const size_t mr = nr * c.pr, mc = nb * c.pc;
  const size_t d = (size_t)k * n * mr + (size_t)k * n * mc  // M, L
                   + mr * mc                                 // T
                   + (size_t)n * k * (c.pr + c.pc)           // B, Phi
                   + 2 * nr + 2 * nb + mr + mc;              // intervals, nodes
  size_t bytes = d * sizeof(double);
  bytes += nr * sizeof(GemmDescG) + nb * sizeof(GemmSegDesc) +
           ((nr + 1) + (nb + 1) + 2 * nb + 2 * FF_XR * nb + 4) * sizeof(int);
  return bytes + 256;
}

size_t ff_bytes_max(int n) {
  size_t b = 0;
  for (int k = 1; k <= KMAX; ++k) b = b > ff_bytes(n, k) ? b : ff_bytes(n, k);
  return b;
}

// Every buffer starts on 16 bytes (pr, pc even) for the products' vector loads.
FarField ff_layout(void* base, int n, int k) {
  const FfCfg c = ff_cfg(k);
  FarField f;
  f.n = n;
  f.k = k;
  f.nb = ff_blocks(n);
  f.nr = n / c.rb;
  f.rb = c.rb;
  f.pr = c.pr;
  f.pc = c.pc;
  f.pad = 0;
  f.etar = c.etar;
  f.etac = c.etac;
  const size_t mr = (size_t)f.nr * c.pr, mc = (size_t)f.nb * c.pc;
  double* d = static_cast<double*>(base);
  f.M = d;
  d += (size_t)k * n * mr;
  f.L = d;
  d += (size_t)k * n * mc;
  f.T = d;
  d += mr * mc;
  f.B = d;
  d += (size_t)n * k * c.pr;
  f.Phi = d;
  d += (size_t)n * k * c.pc;
  f.ivr = d;
  d += 2 * (size_t)f.nr;
  f.ivc = d;
  d += 2 * (size_t)f.nb;
  f.xn = d;
  d += mc;
  f.yn = d;
  d += mr;
  GemmDescG* g = reinterpret_cast<GemmDescG*>(d);
  f.desc = g;
  g += f.nr;
  GemmSegDesc* sg = reinterpret_cast<GemmSegDesc*>(g);
  f.seg = sg;
  sg += f.nb;
  int* ip = reinterpret_cast<int*>(sg);
  f.prefix = ip;
  ip += (f.nr + 1) + (f.nb + 1);
  f.near = ip;
  ip += 2 * f.nb;
  f.extra = ip;
  ip += 2 * FF_XR * f.nb;
  f.flags = ip;
  return f;
}

// Chebyshev node m of P on [lo, hi] (c = ff_cos(m, P)) and its barycentric
// weight.
__device__ __forceinline__ double ff_cos(int m, int P) { return cos((2 * m + 1) * M_PI / (2.0 * P)); }
__device__ __forceinline__ double ff_node(double lo, double hi, double c) {
  return 0.5 * (lo + hi) + 0.5 * (hi - lo) * c;
}
__device__ __forceinline__ double ff_bw(int m, int P) {
  const double s = sin((2 * m + 1) * M_PI / (2.0 * P));
  return (m & 1) ? -s : s;
}

// Lagrange basis S_m(y), m < P, of the nodes nd (second barycentric form;
// bw: the weights ff_bw).
template <int P>
__device__ __forceinline__ void ff_basis(const double* nd, const double* bw, double y,
                                         double* S) {
  int hit = -1;
  double sum = 0.0;
#pragma unroll
  for (int m = 0; m < P; ++m) {
    const double dy = y - nd[m];
    if (dy == 0.0) hit = m;
    S[m] = bw[m] / (dy == 0.0 ? 1.0 : dy);
    sum += S[m];
  }
  if (hit >= 0) {
#pragma unroll
    for (int m = 0; m < P; ++m) S[m] = (m == hit) ? 1.0 : 0.0;
  } else {
    const double r = 1.0 / sum;
#pragma unroll
    for (int m = 0; m < P; ++m) S[m] *= r;
  }
}

// Absolute point at which column p was formed (deflated columns: its eigenvalue).
__device__ __forceinline__ double ff_colx(const Work& w, int p) {
  const ColParam& cp = w.colp[p];
  return cp.drow >= 0 ? w.lam_fin[p] : cp.d_o + cp.tau;
}

// One block per row block: its pole interval; the first nb blocks also take the
// interval of the column points of column block blockIdx.x.
__global__ __launch_bounds__(256) void ff_interval_kernel(Work w, FarField f) {
  __shared__ double s_lo[4], s_hi[4];
  const int J = blockIdx.x, n = w.n;
  if (J < f.nr && threadIdx.x == 0) {
    const int r0 = ff_row_begin(f, J), r1 = ff_row_end(f, J);
    f.ivr[2 * J] = w.lam_in[r0];
    f.ivr[2 * J + 1] = w.lam_in[r1 - 1];
  }
  if (J >= f.nb) return;
  const int c0 = J * FF_B, b = ff_bsize(n, f.nb, J, FF_B);
  double lo = INFINITY, hi = -INFINITY;
  for (int p = c0 + threadIdx.x; p < c0 + b; p += 256) {
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
    f.ivc[2 * J] = s_lo[0];
    f.ivc[2 * J + 1] = s_hi[0];
  }
}

// Column block I and row block h far apart: distance at least etac times the
// column width and etar times the row width (false if any bound is NaN); ivr and
// ivc are the plan's copies of the intervals.
__device__ __forceinline__ bool ff_far(const FarField& f, const double* ivr, const double* ivc,
                                       int I, int h) {
  const double ylo = ivr[2 * h], yhi = ivr[2 * h + 1];
  const double xlo = ivc[2 * I], xhi = ivc[2 * I + 1];
  const double dist = fmax(xlo - yhi, ylo - xhi);
  return dist >= f.etac * (xhi - xlo) && dist >= f.etar * (yhi - ylo);
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

// One block: near rows of every column block, the path decision, nodes,
// descriptors and prefixes.
__global__ __launch_bounds__(256) void ff_plan_kernel(Work w, FarField f) {
  __shared__ int s_ok, s_full, s_lastpos;
  __shared__ int s_sl[FF_MAXNB];     // k-slices of each column block's product
  __shared__ short s_inv[FF_MAXNB];  // column block of each launch position
  // the intervals, read many times by the near-row searches
  __shared__ double s_ivr[2 * (2 * FF_MAXNB + 1)], s_ivc[2 * FF_MAXNB];  // nr <= 2 nb + 1
  __shared__ double s_cr[FF_PMAX], s_cc[FF_PMAX];
  const int n = w.n, k = w.k, nb = f.nb, nr = f.nr;
  const int kpr = k * f.pr, kpc = k * f.pc, rpc = FF_B / f.rb;
  if (threadIdx.x == 0) {
    s_ok = (__builtin_nontemporal_load(&w.st->status) == 0) && (w.info->n_groups == 0);
    s_full = 0;
  }
  if (threadIdx.x < f.pr) s_cr[threadIdx.x] = ff_cos(threadIdx.x, f.pr);
  if (threadIdx.x < f.pc) s_cc[threadIdx.x] = ff_cos(threadIdx.x, f.pc);
  for (int e = threadIdx.x; e < 2 * nr; e += 256) s_ivr[e] = f.ivr[e];
  for (int e = threadIdx.x; e < 2 * nb; e += 256) s_ivc[e] = f.ivc[e];
  __syncthreads();
  for (int h = threadIdx.x; h < nr; h += 256) {
    const double lo = s_ivr[2 * h], hi = s_ivr[2 * h + 1];
    if (!(hi > lo && isfinite(lo) && isfinite(hi))) s_ok = 0;
  }
  for (int I = threadIdx.x; I < nb; I += 256) {
    const double lo = s_ivc[2 * I], hi = s_ivc[2 * I + 1];
    if (!(hi > lo && isfinite(lo) && isfinite(hi))) s_ok = 0;
  }
  __syncthreads();
  for (int I = threadIdx.x; I < nb; I += 256) {
    // the rows within rb of the column block, then widened while the next row
    // block is not far
    int lo = max(0, I * rpc - 1);
    int hi = (I + 1 == nb) ? nr - 1 : min(nr - 1, (I + 1) * rpc);
    int cnt = 0;
    if (s_ok) {
      while (lo > 0 && !ff_far(f, s_ivr, s_ivc, I, lo - 1)) --lo;
      while (hi < nr - 1 && !ff_far(f, s_ivr, s_ivc, I, hi + 1)) ++hi;
      int run = -1;  // first row block of the current range of near blocks
      for (int h = 0; h <= nr; ++h) {
        const bool nh = h < nr && (h < lo || h > hi) && !ff_far(f, s_ivr, s_ivc, I, h);
        if (nh && run < 0) run = h;
        if (!nh && run >= 0) {
          if (cnt < FF_XR) {
            f.extra[2 * (I * FF_XR + cnt)] = run;
            f.extra[2 * (I * FF_XR + cnt) + 1] = h - 1;
          }
          ++cnt;
          run = -1;
        }
      }
    }
    if (cnt > FF_XR) {  // this column block is multiplied exactly over all rows
      cnt = 0;
      lo = 0;
      hi = nr - 1;
    }
    f.near[2 * I] = lo;
    f.near[2 * I + 1] = hi;
    for (int r = cnt; r < FF_XR; ++r) {
      f.extra[2 * (I * FF_XR + r)] = -1;
      f.extra[2 * (I * FF_XR + r) + 1] = -2;
    }
    int rows = ff_row_end(f, hi) - ff_row_begin(f, lo);
    int sl = (rows + 15) / 16 + (kpc + 15) / 16;
    for (int r = 0; r < cnt; ++r) {
      const int m = ff_row_end(f, f.extra[2 * (I * FF_XR + r) + 1]) -
                    ff_row_begin(f, f.extra[2 * (I * FF_XR + r)]);
      rows += m;
      sl += (m + 15) / 16;
    }
    s_sl[I] = sl;
    if (2 * rows >= n) atomicAdd(&s_full, 1);  // half the rows or more exact
  }
  __syncthreads();
  // half or more of the column blocks take half the rows or more exactly: the
  // dense product is cheaper
  if (threadIdx.x == 0 && 2 * s_full >= nb) s_ok = 0;
  __syncthreads();
  const bool ok = s_ok != 0;
  for (int e = threadIdx.x; e < nr * f.pr; e += 256) {
    const int h = e / f.pr;
    f.yn[e] = ok ? ff_node(s_ivr[2 * h], s_ivr[2 * h + 1], s_cr[e % f.pr]) : 0.0;
  }
  for (int e = threadIdx.x; e < nb * f.pc; e += 256) {
    const int I = e / f.pc;
    f.xn[e] = ok ? ff_node(s_ivc[2 * I], s_ivc[2 * I + 1], s_cc[e % f.pc]) : 0.0;
  }
  // P2M: M_h = Q(:, h) B_h
  for (int h = threadIdx.x; h < nr; h += 256) {
    const int r0 = ff_row_begin(f, h), b = ff_row_end(f, h) - r0;
    f.desc[h] = ff_desc(w.Q_in + (size_t)r0 * n, n, f.B + (size_t)r0 * kpr, b,
                        f.M + (size_t)h * f.pr * k * n, n, n, kpr, b, FF_PTILE);
  }
  for (int I = threadIdx.x; I < nb; I += 256) {
    const int b = ff_bsize(n, nb, I, FF_B), c0 = I * FF_B;
    // Q'(:, I) = Q(:, band) W(band, I) + sum_ranges Q(:, R) W(R, I) + L_I Phi_I.
    // Launch order of the column blocks' products: longer ones first, so that
    // their tiles do not run last, alone, after the short ones (stable in I; the
    // tiles compute the same in any order).
    const int mine = s_sl[I];
    int pos = 0;
    for (int J = 0; J < nb; ++J) pos += (s_sl[J] > mine || (s_sl[J] == mine && J < I)) ? 1 : 0;
    s_inv[pos] = (short)I;
    if (I == nb - 1) s_lastpos = pos;
    GemmSegDesc& g = f.seg[pos];  // written in place
    int ns = 0, sl = 0;
    bool vec = !(n & 1) && !(kpc & 1);
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
    auto add_rows = [&](int hlo, int hhi) {
      const int j0 = ff_row_begin(f, hlo);
      add(w.Q_in + (size_t)j0 * n, w.W + (size_t)c0 * n + j0, n, ff_row_end(f, hhi) - j0);
    };
    add_rows(f.near[2 * I], f.near[2 * I + 1]);
    for (int r = 0; r < FF_XR; ++r) {
      const int hlo = ok ? f.extra[2 * (I * FF_XR + r)] : -1;
      if (hlo >= 0) add_rows(hlo, f.extra[2 * (I * FF_XR + r) + 1]);
    }
    add(f.L + (size_t)I * f.pc * k * n, f.Phi + (size_t)c0 * kpc, kpc, kpc);
    for (int r = ns; r < GSEG; ++r) {
      g.A[r] = g.B[r] = nullptr;
      g.lda[r] = g.ldb[r] = g.K[r] = 0;
      g.send[r] = sl;
    }
    g.C = w.Q_out + (size_t)c0 * n;
    g.M = n;
    g.N = b;
    g.ldc = n;
    g.vec = vec && !((uintptr_t)g.C & 15);
    g.tiles_m = ff_tiles(n);
    g.nseg = ns;
  }
  __syncthreads();
  // tile offsets: P2M's are equal per row block; every column block has
  // ff_tiles(FF_B) column tiles but the last, which may have more
  const int tm = ff_tiles(n), pt = ff_ptiles(n) * ff_ptiles(kpr);
  const int extra = ff_tiles(ff_bsize(n, nb, nb - 1, FF_B)) - ff_tiles(FF_B);
  for (int h = threadIdx.x; h <= nr; h += 256) f.prefix[h] = h * pt;
  for (int q = threadIdx.x; q <= nb; q += 256)  // before the q-th product launched
    f.prefix[(nr + 1) + q] = tm * (ff_tiles(FF_B) * q + (s_lastpos < q ? extra : 0));
  if (threadIdx.x == 0) {
    f.flags[0] = ok ? 0 : 1;                                             // far path skipped
    f.flags[1] = (ok || __builtin_nontemporal_load(&w.st->status) != 0) ? 1 : 0;  // dense skipped
  }
}

// T((h, m), (I, l)) = 1/(xhat_{I,l} - yhat_{h,m}) on far pairs, 0 on near ones.
__global__ __launch_bounds__(256) void ff_t_kernel(FarField f) {
  if (__builtin_nontemporal_load(&f.flags[0]) != 0) return;
  const int mr = f.nr * f.pr;
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long long)mr * f.nb * f.pc) return;
  const int col = (int)(e / mr), row = (int)(e % mr);
  f.T[e] = ff_near(f, col / f.pc, row / f.pr) ? 0.0 : 1.0 / (f.xn[col] - f.yn[row]);
}

// Rows: B_h(j, m k + a) = u_{j,a} S_{h,m}(lambda_j).  Columns: Phi((l k + a), p) =
// S_{I,l}(x_p) c_{p,a} (zero for deflated columns).  Threads 0..n-1 take rows,
// n..2n-1 columns.
template <int PR, int PC>
__global__ __launch_bounds__(256) void ff_weights_kernel(Work w, FarField f) {
  __shared__ double s_bwr[PR], s_bwc[PC];
  if (__builtin_nontemporal_load(&f.flags[0]) != 0) return;
  const int n = w.n, k = w.k, nb = f.nb, nr = f.nr;
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (threadIdx.x < PR) s_bwr[threadIdx.x] = ff_bw(threadIdx.x, PR);
  if (threadIdx.x < PC) s_bwc[threadIdx.x] = ff_bw(threadIdx.x, PC);
  __syncthreads();
  if (t >= 2 * n) return;
  if (t < n) {
    double S[PR];
    const int r = t, h = min(r / f.rb, nr - 1), r0 = ff_row_begin(f, h);
    const int j = r - r0, b = ff_row_end(f, h) - r0;
    const int jr = w.rmap[r];
    ff_basis<PR>(f.yn + h * PR, s_bwr, w.lam_in[r], S);
    double* Bh = f.B + (size_t)r0 * k * PR;
    for (int a = 0; a < k; ++a) {
      const double u = jr >= 0 ? w.ru[(size_t)jr * k + a] : 0.0;
#pragma unroll
      for (int m = 0; m < PR; ++m) Bh[(size_t)(m * k + a) * b + j] = u * S[m];
    }
  } else {
    double S[PC];
    const int p = t - n, I = min(p / FF_B, nb - 1);
    const ColParam& cp = w.colp[p];
    ff_basis<PC>(f.xn + I * PC, s_bwc, ff_colx(w, p), S);
    double* ph = f.Phi + (size_t)p * k * PC;
    for (int a = 0; a < k; ++a) {
      const double c = cp.drow >= 0 ? 0.0 : cp.c[a];
#pragma unroll
      for (int l = 0; l < PC; ++l) ph[l * k + a] = S[l] * c;
    }
  }
}

hipError_t launch_ff_plan(const Work& w, const FarField& f, hipStream_t s) {
  if (f.nb < 1 || f.nr < f.nb) return hipErrorInvalidValue;
  hipLaunchKernelGGL(ff_interval_kernel, dim3(f.nr), dim3(256), 0, s, w, f);
  hipLaunchKernelGGL(ff_plan_kernel, dim3(1), dim3(256), 0, s, w, f);
  return hipGetLastError();
}

hipError_t launch_qw_farfield(const Work& w, const FarField& f, hipStream_t s) {
  const int n = w.n, k = w.k, nb = f.nb, nr = f.nr;
  const int mr = nr * f.pr, mc = nb * f.pc;
  if (nb < 1 || nr < nb) return hipErrorInvalidValue;
  const long long ne = (long long)mr * mc;
  hipLaunchKernelGGL(ff_t_kernel, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, f);
  const dim3 wg((2 * n + 255) / 256);
  if (f.pr == 20 && f.pc == 24)
    hipLaunchKernelGGL((ff_weights_kernel<20, 24>), wg, dim3(256), 0, s, w, f);
  else if (f.pr == 20 && f.pc == 20)
    hipLaunchKernelGGL((ff_weights_kernel<20, 20>), wg, dim3(256), 0, s, w, f);
  else
    return hipErrorInvalidValue;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int tm = ff_tiles(n);
  int band = 0;
  for (int I = 0; I < nb; ++I) band += tm * ff_tiles(ff_bsize(n, nb, I, FF_B));
  const int p2m = nr * ff_ptiles(n) * ff_ptiles(k * f.pr);
  // the dense product, used when the plan rejected the far-field path
  e = launch_dgemm(n, n, n, w.Q_in, n, w.W, n, w.Q_out, n, f.flags + 1, s);
  if (e != hipSuccess) return e;
  e = launch_dgemm_desc(false, FF_PTILE, f.desc, f.prefix, nr, p2m, f.flags, s);
  if (e != hipSuccess) return e;
  e = launch_dgemm(k * n, mc, mr, f.M, k * n, f.T, mr, f.L, k * n, f.flags, s);
  if (e != hipSuccess) return e;
  return launch_dgemm_seg(f.seg, f.prefix + (nr + 1), nb, band, f.flags, s);
}

}  // namespace eigupd
