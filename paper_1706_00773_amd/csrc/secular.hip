// secular.hip -- location and refinement of the roots of the multiple-rank
// secular equation det(I - Sigma U^T (xI - D)^{-1} U) = 0 (Sec. 2.1, eq. (1)).
//
// Counting.  For x not a pole, the number of eigenvalues of D + U Sigma U^T
// strictly below x is
//     nu(x) = #{d_j < x} + neg(S(x)) - p,    S(x) = sum_j u_j u_j^T / (x - d_j) - Sigma,
// (inertia of the bordered matrix [[D - xI, U], [U^T, -Sigma]] taken two
// ways).  It is the integer that the paper's modified Sturm chain yields
// (Sec. 2.2) but needs only a k-by-k inertia.  At a pole d_s with rows Y_s:
//     nu(d_s) = #{d_j < d_s} + r_s + neg(P^T T_s P) - p,
// T_s = sum_{j not in s} u_j u_j^T / (d_s - d_j) - Sigma, P an orthonormal
// basis of the complement of the row space of Y_s.  The pole counts give the
// location vector of Sec. 2.2 for any rank: interval t holds
// nu(d_t) - nu(d_{t-1}) roots.
//
// Refinement.  Each root is solved in shifted coordinates x = d_o + tau around
// the nearer pole of its interval; every difference x - d_j is formed as
// tau - (d_j - d_o).  Between poles every eigenvalue branch of S(x) is
// decreasing (S' = -sum u_j u_j^T / (x - d_j)^2), so a root is a simple zero of
// g(x) = (x - d_a)^{r_a} (x - d_b)^{r_b} det S(x), which is smooth on the whole
// interval [d_a, d_b].  Newton steps on g, d log g / dx = r_a/(x - d_a) +
// r_b/(x - d_b) + tr(S^{-1} S'), are taken inside a bracket kept by the count;
// a step that leaves the bracket or does not halve is replaced by bisection
// (the zero finder of Sec. 2.3 with the count deciding the side).  Two or more
// roots in one interval are first separated by count bisection.
//
// Kernel shape.  A block owns RPB roots and WV waves; each wave sums S and S'
// over its slice of the poles for all RPB roots, with the 64/RPB parts of the
// wave taking alternate poles of the slice.  The slice is streamed through a
// per-wave LDS tile (coalesced loads, prefetched one tile ahead into
// registers) and every lane of a part reads the same pole (an LDS broadcast).
// Partial sums meet in LDS, and wave 0 does the k-by-k work (Jacobi
// eigen-decomposition: inertia, Newton step, null vector) and writes the next
// points.
#include <atomic>

#include "common.h"
#include "smallmat.h"

namespace eigupd {

constexpr double EPSU = 1.1102230246251565e-16;  // 2^-53

template <int K>
struct Cfg {
  static constexpr int NS = K * (K + 1) / 2;
  // waves per block: from rank 4 a wave holds one SIMD (above 128 VGPRs), so 4
  // waves fill a CU's SIMDs (2 waves at ranks 5-8 left half of them idle: pole
  // counts and roots 1.5-1.8x slower at n = 8192)
  static constexpr int WV = (K <= 1) ? 16 : (K <= 3) ? 8 : 4;
  static constexpr int RPB = 32;          // roots (or poles) per block
  static constexpr int SPLIT = 64 / RPB;  // parts of a wave sharing one root
  static constexpr int TP = 128;          // poles per LDS tile per wave
};

template <int K, int TP>
struct PoleTile {
  double d[TP];
  double u[TP][K];
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Calls f(r, u) for the poles [jb, je) of this wave, with r = 1/(tau - (d_j - d_o))
// (0 for a pole at distance 0, i.e. x on the pole); part `part` of the wave (of
// SPLIT) takes poles jb + part, jb + part + SPLIT, ...  Tiles of TP poles go
// global -> registers (one tile ahead) -> LDS, and every lane of a part reads the
// same pole.
template <int K, int TP, int SPLIT, int UNR = 2, typename F>
__device__ __forceinline__ void sweep_poles(const double* __restrict__ rd,
                                            const double* __restrict__ ru, int jb, int je,
                                            double tau, double d_o, PoleTile<K, TP>& tile, F&& f) {
  constexpr int PER = TP / 64;
  const int lane = threadIdx.x & 63;
  const int part = lane / (64 / SPLIT);
  double pd[PER], pu[PER][K];
  auto load = [&](int base) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int j = base + p * 64 + lane;
      const bool ok = j < je;
      pd[p] = ok ? rd[j] : 0.0;
#pragma unroll
      for (int c = 0; c < K; ++c) pu[p][c] = ok ? ru[(size_t)j * K + c] : 0.0;
    }
  };
  if (jb < je) load(jb);
  for (int base = jb; base < je; base += TP) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      tile.d[p * 64 + lane] = pd[p];
#pragma unroll
      for (int c = 0; c < K; ++c) tile.u[p * 64 + lane][c] = pu[p][c];
    }
    wave_sync();
    if (base + TP < je) load(base + TP);
    const int cnt = min(TP, je - base);
#pragma unroll UNR
    for (int q = part; q < cnt; q += SPLIT) {
      double u[K];
#pragma unroll
      for (int c = 0; c < K; ++c) u[c] = tile.u[q][c];
      f(recip(tau - (tile.d[q] - d_o)), u);
    }
    wave_sync();
  }
}

// Adds up the partial sums of the SPLIT parts of a wave (every lane gets the total).
template <int SPLIT, int N>
__device__ __forceinline__ void combine_parts(double (&a)[N]) {
#pragma unroll
  for (int off = 32; off >= 64 / SPLIT; off >>= 1)
#pragma unroll
    for (int e = 0; e < N; ++e) a[e] += __shfl_xor(a[e], off, 64);
}

// S = sum_j u_j u_j^T r_j (without -Sigma) over this wave's poles, combined across
// the parts of the wave.
template <int K, int TP, int SPLIT>
__device__ __forceinline__ void sweep(const double* __restrict__ rd, const double* __restrict__ ru,
                                      int jb, int je, double tau, double d_o,
                                      double (&S)[Sym<K>::NS], PoleTile<K, TP>& tile) {
  constexpr int NS = Sym<K>::NS;
#pragma unroll
  for (int e = 0; e < NS; ++e) S[e] = 0.0;
  sweep_poles<K, TP, SPLIT>(rd, ru, jb, je, tau, d_o, tile, [&](double r, const double (&u)[K]) {
    double v[K];
#pragma unroll
    for (int c = 0; c < K; ++c) v[c] = u[c] * r;
#pragma unroll
    for (int a = 0; a < K; ++a)
#pragma unroll
      for (int b = a; b < K; ++b) S[Sym<K>::at(a, b)] = fma(u[a], v[b], S[Sym<K>::at(a, b)]);
  });
  combine_parts<SPLIT>(S);
}

// Pole value written into the unused tail of a tile: with u = 0 it contributes
// nothing, and tau - (PAD_D - d_o) is never 0.
constexpr double PAD_D = 1e300;

// The root solver's tile: the poles and, per pole, ||u_j||^2.
template <int K, int TP>
struct RootTile {
  double d[TP];
  double nrm[TP];
  double u[TP][K];
};

// As sweep(), and also e = sum_j ||u_j||^2 |r_j| (= sum_j sum_a |u_ja v_ja|), the
// size of the terms summed into the diagonal of S, which bounds its rounding
// error; ||u_j||^2 is formed once per tile, not once per root.
// For the root solver only: x is strictly between two poles, so 1/(x - d_j) needs
// no guard, and the pole loop is the same for every lane (the tile tail is padded
// with zero-weight poles), which lets the compiler pipeline the LDS reads.
// r_j takes one Newton step from the hardware estimate (relative error ~1e-15,
// well below the rounding of the sums it enters).
template <int K, int TP, int SPLIT, int UNR = 4>
__device__ __forceinline__ void sweep_err(const double* __restrict__ rd,
                                          const double* __restrict__ ru, int jb, int je,
                                          double tau, double d_o, double (&S)[Sym<K>::NS],
                                          double (&G)[Sym<K>::NS], double& e,
                                          RootTile<K, TP>& tile) {
  static_assert(TP % SPLIT == 0, "a padded tile holds whole rounds");
  constexpr int NS = Sym<K>::NS;
  constexpr int PER = TP / 64;
  const int lane = threadIdx.x & 63;
  const int part = lane / (64 / SPLIT);
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    S[q] = 0.0;
    G[q] = 0.0;
  }
  double acc_e[1] = {0.0};
  double pd[PER], pu[PER][K];
  auto load = [&](int base) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int j = base + p * 64 + lane;
      const bool ok = j < je;
      pd[p] = ok ? rd[j] : PAD_D;
#pragma unroll
      for (int c = 0; c < K; ++c) pu[p][c] = ok ? ru[(size_t)j * K + c] : 0.0;
    }
  };
  if (jb < je) load(jb);
  for (int base = jb; base < je; base += TP) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      double nn = 0.0;
#pragma unroll
      for (int c = 0; c < K; ++c) {
        tile.u[p * 64 + lane][c] = pu[p][c];
        nn = fma(pu[p][c], pu[p][c], nn);
      }
      tile.d[p * 64 + lane] = pd[p];
      tile.nrm[p * 64 + lane] = nn;
    }
    wave_sync();
    if (base + TP < je) load(base + TP);
    const int rounds = (min(TP, je - base) + SPLIT - 1) / SPLIT;
#pragma unroll UNR
    for (int q0 = 0; q0 < rounds; ++q0) {
      const int q = q0 * SPLIT + part;
      double u[K], v[K];
#pragma unroll
      for (int c = 0; c < K; ++c) u[c] = tile.u[q][c];
      const double y = tau - (tile.d[q] - d_o);
      double r = __builtin_amdgcn_rcp(y);
      r = fma(r, fma(-y, r, 1.0), r);
      acc_e[0] = fma(tile.nrm[q], fabs(r), acc_e[0]);
#pragma unroll
      for (int c = 0; c < K; ++c) v[c] = u[c] * r;
#pragma unroll
      for (int a = 0; a < K; ++a) {
#pragma unroll
        for (int b = a; b < K; ++b) {
          S[Sym<K>::at(a, b)] = fma(u[a], v[b], S[Sym<K>::at(a, b)]);
          G[Sym<K>::at(a, b)] = fma(v[a], v[b], G[Sym<K>::at(a, b)]);
        }
      }
    }
    wave_sync();
  }
  combine_parts<SPLIT>(S);
  combine_parts<SPLIT>(G);
  combine_parts<SPLIT>(acc_e);
  e = acc_e[0];
}

// ---------------------------------------------------------------------------
// Pole counts nu(d_s) for every segment s.
// ---------------------------------------------------------------------------
template <int K>
__device__ __forceinline__ void polecount_body(const Work& w, int bid) {
  constexpr int NS = Sym<K>::NS, WV = Cfg<K>::WV, RPB = Cfg<K>::RPB, TP = Cfg<K>::TP;
  __shared__ double s_part[WV][NS][RPB];
  __shared__ PoleTile<K, TP> s_tile[WV];
  if (update_cancelled(w.st)) return;
  if (w.info->loc_alpha) return;  // the residue signs located the roots
  const int n_s = w.info->n_s, n_d = w.info->n_d;
  const int s0 = bid * RPB;
  if (s0 >= n_s) return;
  const int lane = threadIdx.x & 63, slot = lane % RPB;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int s = min(s0 + slot, n_s - 1);
  const int st = w.seg_start[s];
  const double d_s = w.rd[st];
  const int chunk = (n_d + WV - 1) / WV;
  const int jb = min(n_d, wv * chunk), je = min(n_d, jb + chunk);
  double T[NS];
  // tau = 0 at origin d_s: x - d_j = d_s - d_j; rows of segment s give 0 and are skipped
  sweep<K, TP, Cfg<K>::SPLIT>(w.rd, w.ru, jb, je, 0.0, d_s, T, s_tile[wv]);
  if (lane < RPB) {
#pragma unroll
    for (int e = 0; e < NS; ++e) s_part[wv][e][slot] = T[e];
  }
  __syncthreads();
  if (wv != 0 || lane >= RPB || s0 + slot >= n_s) return;
#pragma unroll
  for (int e = 0; e < NS; ++e) {
    double acc = 0.0;
    for (int q = 0; q < WV; ++q) acc += s_part[q][e][slot];
    T[e] = acc;
  }
#pragma unroll
  for (int c = 0; c < K; ++c) T[Sym<K>::at(c, c)] -= ((w.sig_pos_mask >> c) & 1) ? 1.0 : -1.0;
  const int r = max(1, min(w.seg_r[s], K));
  double Y[K][K];
#pragma unroll
  for (int h = 0; h < K; ++h)
#pragma unroll
    for (int c = 0; c < K; ++c) Y[h][c] = w.ru[(size_t)(st + min(h, r - 1)) * K + c];
  const int neg = neg_count_compressed<K>(T, Y, r);
  w.nu[s] = st + r + neg - w.info->p;
}

// ---------------------------------------------------------------------------
// Location: make the pole counts monotone, then give every root its interval.
// ---------------------------------------------------------------------------
constexpr int LNT = 1024;

__device__ __forceinline__ void locate_body(const Work& w) {
  __shared__ int shi[LNT / 64 + 1];
  if (update_cancelled(w.st)) return;
  const int n_s = w.info->n_s, n_d = w.info->n_d;
  // running maximum, clamped to [0, n_d] (0 is the identity: the clamped counts
  // are >= 0): each thread takes one run of consecutive counts, the runs' maxima
  // are scanned across the block, then each run is written.  Runs of up to
  // LRUN counts are held in registers, their loads issued together.
  constexpr int LRUN = 16;
  const int per = (n_s + LNT - 1) / LNT;
  const int b0 = min(n_s, (int)threadIdx.x * per), b1 = min(n_s, b0 + per);
  auto count = [&](int s) { return min(max(w.nu[s], 0), n_d); };
  const bool in_regs = per <= LRUN;  // the same for every thread
  int x[LRUN];
  int run = 0;
  if (in_regs) {
#pragma unroll
    for (int e = 0; e < LRUN; ++e) x[e] = (b0 + e < b1) ? count(b0 + e) : 0;
#pragma unroll
    for (int e = 0; e < LRUN; ++e) run = max(run, x[e]);
  } else {
    for (int s = b0; s < b1; ++s) run = max(run, count(s));
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int v = run;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(v, off, 64);
    if (lane >= off) v = max(v, t);
  }
  if (lane == 63) shi[wv] = v;
  __syncthreads();
  int pre = __shfl_up(v, 1, 64);  // the maximum over the runs of lower lanes
  if (lane == 0) pre = 0;
  for (int q = 0; q < wv; ++q) pre = max(pre, shi[q]);
  if (in_regs) {
#pragma unroll
    for (int e = 0; e < LRUN; ++e) {
      pre = max(pre, x[e]);
      if (b0 + e < b1) w.nu[b0 + e] = pre;
    }
  } else {
    for (int s = b0; s < b1; ++s) {
      pre = max(pre, count(s));
      w.nu[s] = pre;
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t <= n_s; t += LNT) {
    const int lo = (t == 0) ? 0 : w.nu[t - 1];
    const int hi = (t == n_s) ? n_d : w.nu[t];
    for (int i = lo; i < hi; ++i) {
      w.root_t[i] = t;
      w.root_clo[i] = lo;
      w.root_chi[i] = hi;
    }
  }
}

// ---------------------------------------------------------------------------
// Root refinement.
// ---------------------------------------------------------------------------
enum { PH_FIRST = 0, PH_SOLVE = 1, PH_DONE = 2 };

// Newton steps below STAG |tau| that no longer halve have reached the rounding
// floor of the secular sums; the iteration stops there.  Near a pole that floor
// can lie far above STAG |tau| (the evaluation of S loses relative accuracy in
// tau there); it is recognised directly: Newton no longer halving while the
// smallest |eigenvalue| of S is below NOISE_C eps times the size of the terms
// summed into its diagonal.
constexpr double STAG = 1e-9;
constexpr double NOISE_C = 64.0;
// Newton in its quadratic phase: a step at most QUAD_R times the previous one.
// Then the next step is about r^2 times this one (r the ratio of the two), and
// when that is below the rounding level of tau the Newton point is taken
// without another evaluation.
constexpr double QUAD_R = 1e-3;

#ifndef ROWS_MIN_K
#define ROWS_MIN_K 8
#endif

// Launch shape of the root solver: RPB root slots per block, each slot's pole
// sums split over WV waves x SPLIT parts of a wave.  A slot whose root has
// converged takes the next unsolved root of the update (a counter in DevInfo),
// so a block runs until the update's roots run out rather than until the
// slowest of a fixed set of roots has converged.
template <int K>
struct RsCfg {
  static constexpr int WV = Cfg<K>::WV;
  static constexpr int RPB = 8;
  static constexpr int SPLIT = 64 / RPB;
  static constexpr int TP = Cfg<K>::TP;
  static constexpr int UNR = 4;
};

// The state of the root held by one solver slot.  It lives in LDS between
// evaluations, so that the pole sweep, which every wave runs, keeps only its own
// accumulators in registers.
struct SlotState {
  double a, b, ra, rb;          // interval ends (pole values) and their multiplicities
  double tlo, thi, tau, d_o;    // bracket and iterate, offsets from the origin pole d_o
  double dxold, dprev;          // previous step sizes
  int i, phase, t, clo, chi;    // root, stage, interval, counts at the bracket ends
  int evals, rows_below, o_seg;
  int two_sided, last_newton;
  int it_min, it_max;           // statistics over the roots this slot has solved
  long long it_sum;
};

template <int K>
__device__ __forceinline__ void rootsolve_body(const Work& w) {
  constexpr int NS = Sym<K>::NS, WV = RsCfg<K>::WV, RPB = RsCfg<K>::RPB, TP = RsCfg<K>::TP;
  constexpr int SPLIT = RsCfg<K>::SPLIT;
  constexpr int KV = (K >= ROWS_MIN_K) ? K : 1;  // eigenvectors of the lane-group solve
  __shared__ double s_part[WV][2 * NS + 1][RPB];
  __shared__ RootTile<K, TP> s_tile[WV];
  __shared__ double s_V[RPB][KV][KV];
  __shared__ SlotState s_st[RPB];
  __shared__ double s_tau[RPB], s_do[RPB];
  __shared__ int s_any;
  if (update_cancelled(w.st)) return;
  const int n_d = w.info->n_d, n_s = w.info->n_s;
  const int r_lo = w.info->r_lo, r_hi = w.info->r_hi;  // the roots to solve
  if (r_lo >= r_hi) return;
  const int lane = threadIdx.x & 63, slot = lane % RPB;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int chunk = (n_d + WV - 1) / WV;
  const int jb = min(n_d, wv * chunk), je = min(n_d, jb + chunk);
  const bool owner = (wv == 0) && (lane < RPB);  // lane `slot` of wave 0 steers slot `slot`

  // takes the next root of the update into the slot (or retires the slot)
  auto start = [&](SlotState& z) {
    z.i = r_lo + atomicAdd(&w.info->root_next, 1);
    if (z.i >= r_hi) {
      z.phase = PH_DONE;
      return;
    }
    z.phase = PH_FIRST;
    z.evals = 0;
    z.dprev = INFINITY;
    z.last_newton = 0;
    z.a = z.b = z.ra = z.rb = 0.0;
    const int t = min(max(w.root_t[z.i], 0), n_s);
    z.t = t;
    z.clo = w.root_clo[z.i];
    z.chi = w.root_chi[z.i];
    z.rows_below = w.seg_start[t];  // rows strictly below any x inside interval t
    const bool has_a = t > 0, has_b = t < n_s;
    z.two_sided = has_a && has_b;
    if (has_a) {
      z.a = w.rd[w.seg_start[t - 1]];
      z.ra = (double)w.seg_r[t - 1];
    }
    if (has_b) {
      z.b = w.rd[w.seg_start[t]];
      z.rb = (double)w.seg_r[t];
    }
    if (z.two_sided) {
      z.o_seg = t - 1;
      z.d_o = z.a;
      z.tlo = 0.0;
      z.thi = z.b - z.a;
      z.tau = 0.5 * z.thi;
    } else if (has_a) {  // right of the last pole
      z.o_seg = t - 1;
      z.d_o = z.a;
      z.tlo = 0.0;
      z.thi = w.info->upper - z.a;
      z.tau = 0.5 * z.thi;
    } else {  // left of the first pole
      z.o_seg = t;
      z.d_o = z.b;
      z.tlo = w.info->lower - z.b;
      z.thi = 0.0;
      z.tau = 0.5 * z.tlo;
    }
    z.dxold = z.thi - z.tlo;
  };
  if (owner) {
    SlotState z;
    z.it_min = 0x7fffffff;
    z.it_max = 0;
    z.it_sum = 0;
    z.tau = z.d_o = 0.0;
    start(z);
    s_st[slot] = z;
    s_tau[slot] = z.tau;
    s_do[slot] = z.d_o;
  }
  if (wv == 0) {
    const unsigned long long live = __ballot(owner && s_st[slot].phase != PH_DONE);
    if (lane == 0) s_any = (live != 0ull);
  }
  __syncthreads();
  if (!s_any) return;

  for (;;) {
    {
      double S[NS], G[NS], err;
      sweep_err<K, TP, SPLIT, RsCfg<K>::UNR>(w.rd, w.ru, jb, je, s_tau[slot], s_do[slot], S, G,
                                             err, s_tile[wv]);
      if (lane < RPB) {
#pragma unroll
        for (int e = 0; e < NS; ++e) {
          s_part[wv][e][slot] = S[e];
          s_part[wv][NS + e][slot] = G[e];
        }
        s_part[wv][2 * NS][slot] = err;
      }
    }
    __syncthreads();
    if (wv == 0) {
      // S(x) = V diag(theta) V^T: the inertia of S, its smallest |theta|, and
      // tr(S^{-1} S') = -sum_m v_m^T G v_m / theta_m.  Ranks >= 5 solve the k x k
      // problem on a group of 8 lanes per slot (lane l: row l), lower ranks on
      // one lane per slot.
      constexpr bool ROWS = (K >= ROWS_MIN_K);
      const int es = ROWS ? (lane >> 3) : slot;
      const bool eowner = ROWS ? ((lane & 7) == 0) : (lane < RPB);
      const bool elive = s_st[es].phase != PH_DONE;
      int neg = 0;
      double phi = 0.0, thmin = INFINITY;
      double err = (double)K;  // the -Sigma diagonal
#pragma unroll 1
      for (int q = 0; q < WV; ++q) err += s_part[q][2 * NS][es];
      if constexpr (ROWS) {
        const int l = lane & 7;
        double a[K], v[K];
#pragma unroll
        for (int c = 0; c < K; ++c) {
          double x = 0.0;
          if (l < K) {
            for (int q = 0; q < WV; ++q) x += s_part[q][Sym<K>::at(l, c)][es];
            if (c == l) x -= ((w.sig_pos_mask >> c) & 1) ? 1.0 : -1.0;
          }
          a[c] = x;
        }
        // the totals of G into wave 0's row of s_part (entries striped over the group)
        for (int e = l; e < NS; e += 8) {
          double g = 0.0;
          for (int q = 0; q < WV; ++q) g += s_part[q][NS + e][es];
          s_part[0][NS + e][es] = g;
        }
        jacobi_eig_rows<K, true>(a, v, elive);
        const double th = (l < K) ? row_at<K>(a, l) : 0.0;
        if (l < K) {
#pragma unroll
          for (int c = 0; c < K; ++c) s_V[es][l][c] = v[c];
        }
        wave_sync();
        // lane m < K: the eigenvector v_m of theta_m is column m of V
        double term = 0.0;
        if (l < K) {
          double col[K];
#pragma unroll
          for (int r = 0; r < K; ++r) col[r] = s_V[es][r][l];
          double vgv = 0.0;
#pragma unroll
          for (int p2 = 0; p2 < K; ++p2) {
            double gv = 0.0;
#pragma unroll
            for (int q2 = 0; q2 < K; ++q2) gv += s_part[0][NS + Sym<K>::at(p2, q2)][es] * col[q2];
            vgv += col[p2] * gv;
          }
          term = -vgv / th;
        }
        phi = group8_sum(term);
        neg = group8_sum_int((l < K && th < 0.0) ? 1 : 0);
        thmin = group8_min((l < K) ? fabs(th) : INFINITY);
      } else if (eowner && elive) {
        double S[NS], G[NS];
#pragma unroll
        for (int e = 0; e < NS; ++e) S[e] = G[e] = 0.0;
#pragma unroll 1
        for (int q = 0; q < WV; ++q) {
#pragma unroll
          for (int e = 0; e < NS; ++e) {
            S[e] += s_part[q][e][es];
            G[e] += s_part[q][NS + e][es];
          }
        }
#pragma unroll
        for (int c = 0; c < K; ++c)
          S[Sym<K>::at(c, c)] -= ((w.sig_pos_mask >> c) & 1) ? 1.0 : -1.0;
        if constexpr (K >= 5) {
          // G rotated along with S: on return G holds V^T G V
          jacobi_eig_congruent<K>(S, G);
#pragma unroll
          for (int m = 0; m < K; ++m) {
            const double th = S[Sym<K>::at(m, m)];
            neg += (th < 0.0) ? 1 : 0;
            thmin = fmin(thmin, fabs(th));
            phi -= G[Sym<K>::at(m, m)] / th;
          }
        } else {
          double V[K][K];
          jacobi_eig<K, true>(S, V);
#pragma unroll
          for (int m = 0; m < K; ++m) {
            const double th = S[Sym<K>::at(m, m)];
            neg += (th < 0.0) ? 1 : 0;
            thmin = fmin(thmin, fabs(th));
            double vgv = 0.0;
#pragma unroll
            for (int p2 = 0; p2 < K; ++p2) {
              double gv = 0.0;
#pragma unroll
              for (int q2 = 0; q2 < K; ++q2) gv += G[Sym<K>::at(p2, q2)] * V[q2][m];
              vgv += V[p2][m] * gv;
            }
            phi -= vgv / th;
          }
        }
      }
      bool live = false;
      if (eowner && elive) {
        SlotState z = s_st[es];
        ++z.evals;
        const int tgt = z.i + 1;
        const int cnt = z.rows_below + neg - w.info->p;
        // d log g / dx = ra/(x-a) + rb/(x-b) + tr(S^{-1} S'); the Newton step is -1/that
        double da, db;
        if (z.o_seg == z.t - 1) {
          da = z.tau;
          db = z.tau - (z.b - z.a);
        } else {
          da = z.tau + (z.b - z.a);
          db = z.tau;
        }
        if (z.ra > 0.0) phi += z.ra / da;
        if (z.rb > 0.0) phi += z.rb / db;
        const double delta = -1.0 / phi;
        if (z.phase == PH_FIRST) {
          z.phase = PH_SOLVE;
          if (z.two_sided && cnt < tgt) {
            // the root lies in the right half: move the origin to b
            z.o_seg = z.t;
            z.d_o = z.b;
            const double gap = z.b - z.a;
            z.tau -= gap;
            z.tlo -= gap;
            z.thi = 0.0;
          }
        }
        if (cnt >= tgt) {
          z.thi = z.tau;
          z.chi = cnt;
        } else {
          z.tlo = z.tau;
          z.clo = cnt;
        }
        const double width = z.thi - z.tlo;
        const double mid = z.tlo + 0.5 * width;
        const bool isolated = (z.clo == tgt - 1) && (z.chi == tgt);
        double next = mid;
        bool conv = false;
        if (width <= 4.0 * EPSU * fmax(fabs(z.tlo), fabs(z.thi))) {
          conv = true;
        } else if (isolated && isfinite(delta)) {
          const double tn = z.tau + delta;
          const double ad = fabs(delta);
          // converged: a step at the rounding level of tau; or Newton no longer
          // halving while its step is small, or while S is singular to within the
          // rounding error of its sums (the noise floor of the evaluation)
          const bool stalled = ad > 0.5 * fabs(z.dprev);
          const double r = ad / fabs(z.dprev);
          const bool quad = z.last_newton && r <= QUAD_R && r * r * ad <= 4.0 * EPSU * fabs(tn) &&
                            tn > z.tlo && tn < z.thi;
          if (ad <= 4.0 * EPSU * fabs(tn) || quad || (stalled && ad <= STAG * fabs(tn)) ||
              (stalled && thmin <= NOISE_C * EPSU * err)) {
            conv = true;
            next = fmin(fmax(tn, z.tlo), z.thi);
          } else if (tn > z.tlo && tn < z.thi && (!z.last_newton || ad <= 0.5 * fabs(z.dxold))) {
            // an in-bracket Newton step is taken unless the previous step was one
            // too and this one does not halve it
            z.dxold = delta;
            next = tn;
          } else {
            z.dxold = 0.5 * width;
          }
          z.dprev = delta;
        }
        z.last_newton = !conv && (next != mid);
        if (!conv && z.evals >= w.max_evals) {
          conv = true;
          atomicOr(&w.st->status, ST_NOCONV);
        }
        if (!conv && !(next > z.tlo && next < z.thi)) next = mid;
        if (next == 0.0) next = (z.tlo == 0.0) ? z.thi : z.tlo;
        z.tau = next;
        if (conv) {
          w.root_o[z.i] = z.o_seg;
          w.root_tau[z.i] = z.tau;
          w.root_clo[z.i] = z.clo;
          w.root_chi[z.i] = z.chi;
          w.root_it[z.i] = z.evals;
          z.it_min = min(z.it_min, z.evals);
          z.it_max = max(z.it_max, z.evals);
          z.it_sum += z.evals;
          start(z);
        }
        s_st[es] = z;
        s_tau[es] = z.tau;
        s_do[es] = z.d_o;
        live = z.phase != PH_DONE;
      }
      const unsigned long long any = __ballot(live);
      if (lane == 0) s_any = (any != 0ull);
    }
    __syncthreads();
    if (!s_any) break;
  }
  if (owner && s_st[slot].it_max > 0) {
    const SlotState& z = s_st[slot];
    atomicMin(&w.info->it_min, z.it_min);
    atomicMax(&w.info->it_max, z.it_max);
    atomicAdd((unsigned long long*)&w.info->it_sum, (unsigned long long)z.it_sum);
  }
}

// ---------------------------------------------------------------------------
// Null vectors at the converged roots (Sec. 2.4).  c is the eigenvector of the
// smallest-magnitude eigenvalue of S(lambda'), scaled so that the eigenvector
// w = (lambda' I - D)^{-1} U c has unit norm.  The norm is summed explicitly,
// ||w||^2 = sum_j (u_j^T c)^2 / (lambda' - d_j)^2 with each dot product formed
// first (near a pole the quadratic form c^T G c would cancel).
//
// A cluster -- consecutive roots of one pole interval whose offsets agree to
// CLUSTER_TOL -- is a multiple (or numerically multiple) eigenvalue: its null
// vectors are not determined one by one.  All its roots are solved at the point
// of its first root: the m smallest-magnitude eigenvectors of S are made
// orthonormal in the inner product of the w's (Gram matrix summed the same
// way), and a Rayleigh-Ritz step separates them: for G-orthonormal C,
// W^T (D + U Sigma U^T) W = x I + C^T (S Sigma S + S) C, a k-by-k quantity.
// Root number pos of the cluster takes the Ritz vector of rank pos.
// ---------------------------------------------------------------------------
constexpr double CLUSTER_TOL = 1e-8;

// Ranks from RV_ROWS_MIN_K up solve rootvec's k x k problems on groups of 8 lanes
// (one row of the matrix per lane), as the root solver does from ROWS_MIN_K up.
#ifndef RV_ROWS_MIN_K
#define RV_ROWS_MIN_K 6
#endif

// The end of rootvec on groups of 8 lanes: every lane of the block calls it once
// the Gram sums of the candidates are in s_part.  Slots whose root is simple
// normalise their first candidate (one lane per slot); the slots of a cluster
// orthonormalise the candidates in the Gram inner product (one lane per slot,
// the coefficient vectors X in LDS) and then take the Ritz vector of their rank
// from the eigenpairs of the k x k Rayleigh quotient H, solved on the lane groups.
// X and H of slot s overwrite the partial sums of slot s in s_part once they
// have been added up.
template <int K, int WV, int RPB>
__device__ __forceinline__ void rootvec_finish_rows(const Work& w, int i0, int r_hi,
                                                    double (&s_part)[WV][2 * Sym<K>::NS][RPB],
                                                    double (&s_C)[K][K][RPB],
                                                    double (&s_th)[K][RPB],
                                                    const double (&s_tau)[RPB],
                                                    const int (&s_mc)[RPB],
                                                    const int (&s_pos)[RPB], int cluster) {
  constexpr int NS = Sym<K>::NS;
  static_assert(K * K <= 2 * NS && WV >= 2, "X and H fit in a slot's partial sums");
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int slot = lane % RPB;
  const bool owner = (wv == 0) && (lane < RPB);
  if (owner && i0 + slot < r_hi) {
    const int i = i0 + slot;
    double gram[NS];
#pragma unroll
    for (int e = 0; e < NS; ++e) {
      double as = 0.0;
      for (int q = 0; q < WV; ++q) as += s_part[q][e][slot];
      gram[e] = as;
    }
    const int m_c = min(s_mc[slot], K);
    if (m_c == 1) {
      const double inv = (gram[0] > 0.0) ? 1.0 / sqrt(gram[0]) : 0.0;
#pragma unroll
      for (int c = 0; c < K; ++c) w.root_c[(size_t)i * K + c] = s_C[0][c][slot] * inv;
      w.root_tv[i] = s_tau[slot];
    } else {
      // Gram-Schmidt of the m_c candidates in the Gram inner product, on
      // coefficient vectors (candidate a is e_a); rows r >= m_c stay zero
      auto X = [&](int r, int a) -> double& { return s_part[0][r * K + a][slot]; };
      auto quadx = [&](const double (&B)[NS], int r1, int r2) {
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < K; ++a) {
          double t = 0.0;
#pragma unroll
          for (int b = 0; b < K; ++b) t += B[Sym<K>::at(a, b)] * X(r2, b);
          acc += X(r1, a) * t;
        }
        return acc;
      };
#pragma unroll 1
      for (int r = 0; r < K; ++r)
#pragma unroll
        for (int a = 0; a < K; ++a) X(r, a) = (r == a && r < m_c) ? 1.0 : 0.0;
#pragma unroll 1
      for (int r = 0; r < m_c; ++r) {
#pragma unroll 1
        for (int l2 = 0; l2 < r; ++l2) {
          const double g = quadx(gram, l2, r);
#pragma unroll
          for (int a = 0; a < K; ++a) X(r, a) -= g * X(l2, a);
        }
        const double nn = sqrt(fmax(quadx(gram, r, r), 0.0));
        const double inv = (nn > 0.0) ? 1.0 / nn : 0.0;
#pragma unroll
        for (int a = 0; a < K; ++a) X(r, a) *= inv;
      }
      // Rayleigh-Ritz: in candidate coordinates S acts as diag(theta), so
      // C^T (S Sigma S + S) C = Theta (Cc^T Sigma Cc) Theta + Theta
      double Hc[NS];
      double hscale = 0.0;
#pragma unroll
      for (int a = 0; a < K; ++a) {
        hscale = fmax(hscale, fabs(s_th[a][slot]));
#pragma unroll
        for (int b = a; b < K; ++b) {
          double m = 0.0;
#pragma unroll
          for (int c = 0; c < K; ++c)
            m += s_C[a][c][slot] * (((w.sig_pos_mask >> c) & 1) ? 1.0 : -1.0) * s_C[b][c][slot];
          Hc[Sym<K>::at(a, b)] =
              s_th[a][slot] * m * s_th[b][slot] + ((a == b) ? s_th[a][slot] : 0.0);
        }
      }
#pragma unroll 1
      for (int r = 0; r < K; ++r)
#pragma unroll 1
        for (int q = r; q < K; ++q) {
          double acc = (r == q) ? 4.0 * hscale + 1.0 : 0.0;
          if (r < m_c && q < m_c) acc = quadx(Hc, r, q);
          s_part[1][Sym<K>::at(r, q)][slot] = acc;
        }
    }
  }
  if (!cluster) return;
  __syncthreads();
  // the eigenpairs of H on the lane groups, and the Ritz vector of rank pos
  const int l = lane & 7;
#pragma unroll 1
  for (int pass = 0; pass < RPB / (8 * WV); ++pass) {
    const int gs = (pass * WV + wv) * 8 + (lane >> 3);
    const int m_c = min(s_mc[gs], K);
    const bool live = (i0 + gs < r_hi) && m_c > 1;
    if (__ballot(live) == 0ull) continue;
    double a[K], v[K];
#pragma unroll
    for (int c = 0; c < K; ++c) a[c] = (live && l < K) ? s_part[1][Sym<K>::at(l, c)][gs] : 0.0;
    jacobi_eig_rows<K, true>(a, v, live);
    const double hv = row_at<K>(a, l);
    const int pos = min(max(s_pos[gs], 0), m_c - 1);
    double y = 0.0;  // Y(l, m*), m* the eigenvector of ascending rank pos
#pragma unroll
    for (int m = 0; m < K; ++m) {
      const double hm = __shfl(hv, (lane & ~7) + m, 64);
      int rk = 0;
#pragma unroll
      for (int m2 = 0; m2 < K; ++m2) {
        const double h2 = __shfl(hv, (lane & ~7) + m2, 64);
        rk += (h2 < hm || (h2 == hm && m2 < m)) ? 1 : 0;
      }
      if (rk == pos) y = v[m];
    }
    // z = sum_r Y(r, m*) X(r, :) over the group, then this lane's entry of C z
    double out = 0.0;
#pragma unroll
    for (int a2 = 0; a2 < K; ++a2) {
      const double za = group8_sum((live && l < K) ? y * s_part[0][l * K + a2][gs] : 0.0);
      out = fma(za, (l < K) ? s_C[a2][l][gs] : 0.0, out);
    }
    if (live && l < K) {
      const int i = i0 + gs;
      w.root_c[(size_t)i * K + l] = out;
      if (l == 0) w.root_tv[i] = s_tau[gs];
    }
  }
}

template <int K>
__device__ __forceinline__ void rootvec_body(const Work& w, int bid) {
  constexpr int NS = Sym<K>::NS, WV = Cfg<K>::WV, RPB = Cfg<K>::RPB, TP = Cfg<K>::TP;
  constexpr int SPLIT = Cfg<K>::SPLIT;
  constexpr bool ROWS = (K >= RV_ROWS_MIN_K);
  static_assert(!ROWS || (RPB % (8 * WV)) == 0, "whole passes of lane groups");
  __shared__ double s_part[WV][2 * NS][RPB];
  __shared__ PoleTile<K, TP> s_tile[WV];
  __shared__ double s_C[K][K][RPB];
  __shared__ double s_th[K][RPB];
  __shared__ double s_tau[RPB], s_do[RPB];
  __shared__ int s_mc[RPB], s_pos[RPB], s_cluster;
  if (update_cancelled(w.st)) return;
  const int n_d = w.info->n_d, n_s = w.info->n_s;
  const int r_lo = w.info->r_lo, r_hi = w.info->r_hi;  // the solved roots
  const int i0 = r_lo + bid * RPB;
  if (i0 >= r_hi) return;
  const int lane = threadIdx.x & 63, slot = lane % RPB;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int chunk = (n_d + WV - 1) / WV;
  const int jb = min(n_d, wv * chunk), je = min(n_d, jb + chunk);
  const bool owner = (wv == 0) && (lane < RPB);
  const int i = min(i0 + slot, r_hi - 1);
  if (owner) {
    // the cluster [cs, ce) around root i
    const int oi = w.root_o[i], ti = w.root_t[i];
    auto close = [&](int a, int b) {
      const double ta = w.root_tau[a], tb = w.root_tau[b];
      return w.root_o[a] == oi && w.root_o[b] == oi && w.root_t[a] == ti && w.root_t[b] == ti &&
             fabs(ta - tb) <= CLUSTER_TOL * fmax(fabs(ta), fabs(tb));
    };
    int cs = i, ce = i + 1;
    for (int j = i - 1; j >= max(r_lo, i - (K - 1)); --j) {
      if (!close(j, j + 1)) break;
      cs = j;
    }
    for (int j = i + 1; j < min(r_hi, cs + K); ++j) {
      if (!close(j - 1, j)) break;
      ce = j + 1;
    }
    const int m_c = (i0 + slot < r_hi) ? ce - cs : 1;
    s_mc[slot] = m_c;
    s_pos[slot] = i - cs;
    s_tau[slot] = w.root_tau[cs];
    s_do[slot] = w.rd[w.seg_start[min(max(oi, 0), n_s - 1)]];
    const unsigned long long multi = __ballot(m_c > 1);
    if (lane == 0) s_cluster = (multi != 0ull);
  }
  __syncthreads();
  const double tau = s_tau[slot], d_o = s_do[slot];
  {
    double S[NS];
    sweep<K, TP, SPLIT>(w.rd, w.ru, jb, je, tau, d_o, S, s_tile[wv]);
    if (lane < RPB) {
#pragma unroll
      for (int e = 0; e < NS; ++e) s_part[wv][e][slot] = S[e];
    }
  }
  __syncthreads();
  if constexpr (ROWS) {
    // the eigenpairs of S for every slot, on groups of 8 lanes (lane l: row l);
    // each wave takes 8 slots per pass
    const int l = lane & 7;
#pragma unroll 1
    for (int pass = 0; pass < RPB / (8 * WV); ++pass) {
      const int gs = (pass * WV + wv) * 8 + (lane >> 3);
      double a[K], v[K];
#pragma unroll
      for (int c = 0; c < K; ++c) {
        double x = 0.0;
        if (l < K) {
          for (int q = 0; q < WV; ++q) x += s_part[q][Sym<K>::at(l, c)][gs];
          if (c == l) x -= ((w.sig_pos_mask >> c) & 1) ? 1.0 : -1.0;
        }
        a[c] = x;
      }
      jacobi_eig_rows<K, true>(a, v, i0 + gs < r_hi);
      // candidates: eigenvectors of S ordered by |theta| ascending (column m of V
      // is spread over the group: this lane holds its entry l)
      const double th = row_at<K>(a, l);
      double ths[K];
#pragma unroll
      for (int m = 0; m < K; ++m) ths[m] = __shfl(th, (lane & ~7) + m, 64);
      if (l < K) {
#pragma unroll
        for (int m = 0; m < K; ++m) {
          const double am = fabs(ths[m]);
          int rk = 0;
#pragma unroll
          for (int m2 = 0; m2 < K; ++m2) {
            const double a2 = fabs(ths[m2]);
            rk += (a2 < am || (a2 == am && m2 < m)) ? 1 : 0;
          }
          s_C[rk][l][gs] = v[m];
          if (l == m) s_th[rk][gs] = ths[m];
        }
      }
    }
  } else if (owner) {
    double S[NS];
#pragma unroll
    for (int e = 0; e < NS; ++e) {
      double as = 0.0;
      for (int q = 0; q < WV; ++q) as += s_part[q][e][slot];
      S[e] = as;
    }
#pragma unroll
    for (int c = 0; c < K; ++c) S[Sym<K>::at(c, c)] -= ((w.sig_pos_mask >> c) & 1) ? 1.0 : -1.0;
    double V[K][K];
    jacobi_eig<K, true>(S, V);
    // candidates: eigenvectors of S ordered by |theta| ascending
#pragma unroll
    for (int m = 0; m < K; ++m) {
      const double am = fabs(S[Sym<K>::at(m, m)]);
      int rk = 0;
#pragma unroll
      for (int m2 = 0; m2 < K; ++m2) {
        const double a2 = fabs(S[Sym<K>::at(m2, m2)]);
        rk += (a2 < am || (a2 == am && m2 < m)) ? 1 : 0;
      }
#pragma unroll
      for (int c = 0; c < K; ++c) s_C[rk][c][slot] = V[c][m];
      s_th[rk][slot] = S[Sym<K>::at(m, m)];
    }
  }
  __syncthreads();
  // second pass: Gram matrix of the candidates' eigenvectors (just ||w||^2 when
  // the block holds no cluster)
  double gram[NS];
#pragma unroll
  for (int e = 0; e < NS; ++e) gram[e] = 0.0;
  if (!s_cluster) {
    double c0[K];
#pragma unroll
    for (int c = 0; c < K; ++c) c0[c] = s_C[0][c][slot];
    sweep_poles<K, TP, SPLIT>(w.rd, w.ru, jb, je, tau, d_o, s_tile[wv],
                              [&](double r, const double (&u)[K]) {
                                double z = 0.0;
#pragma unroll
                                for (int c = 0; c < K; ++c) z = fma(u[c], c0[c], z);
                                z *= r;
                                gram[0] = fma(z, z, gram[0]);
                              });
  } else if constexpr (ROWS) {
    // the candidates stay in LDS (k^2 coefficients per lane would not fit in
    // registers next to the Gram sums)
    sweep_poles<K, TP, SPLIT, 1>(w.rd, w.ru, jb, je, tau, d_o, s_tile[wv],
                              [&](double r, const double (&u)[K]) {
                                // an opaque slot index: the candidates are read
                                // per pole, not hoisted out of the loop
                                int sl = slot;
                                asm volatile("" : "+v"(sl));
                                double z[K];
#pragma unroll
                                for (int a = 0; a < K; ++a) {
                                  double t = 0.0;
#pragma unroll
                                  for (int c = 0; c < K; ++c) t = fma(u[c], s_C[a][c][sl], t);
                                  z[a] = t * r;
                                }
#pragma unroll
                                for (int a = 0; a < K; ++a)
#pragma unroll
                                  for (int b = a; b < K; ++b)
                                    gram[Sym<K>::at(a, b)] =
                                        fma(z[a], z[b], gram[Sym<K>::at(a, b)]);
                              });
  } else {
    double Cm[K][K];
#pragma unroll
    for (int a = 0; a < K; ++a)
#pragma unroll
      for (int c = 0; c < K; ++c) Cm[a][c] = s_C[a][c][slot];
    sweep_poles<K, TP, SPLIT>(w.rd, w.ru, jb, je, tau, d_o, s_tile[wv],
                              [&](double r, const double (&u)[K]) {
                                double z[K];
#pragma unroll
                                for (int a = 0; a < K; ++a) {
                                  double t = 0.0;
#pragma unroll
                                  for (int c = 0; c < K; ++c) t = fma(u[c], Cm[a][c], t);
                                  z[a] = t * r;
                                }
#pragma unroll
                                for (int a = 0; a < K; ++a)
#pragma unroll
                                  for (int b = a; b < K; ++b)
                                    gram[Sym<K>::at(a, b)] =
                                        fma(z[a], z[b], gram[Sym<K>::at(a, b)]);
                              });
  }
  combine_parts<SPLIT>(gram);
  __syncthreads();
  if (lane < RPB) {
#pragma unroll
    for (int e = 0; e < NS; ++e) s_part[wv][e][slot] = gram[e];
  }
  __syncthreads();
  if constexpr (ROWS) {
    rootvec_finish_rows<K, WV, RPB>(w, i0, r_hi, s_part, s_C, s_th, s_tau, s_mc, s_pos,
                                    s_cluster);
    return;
  }
  if (!owner || i0 + slot >= r_hi) return;
#pragma unroll
  for (int e = 0; e < NS; ++e) {
    double as = 0.0;
    for (int q = 0; q < WV; ++q) as += s_part[q][e][slot];
    gram[e] = as;
  }
  const int m_c = min(s_mc[slot], K);
  const int pos = min(max(s_pos[slot], 0), m_c - 1);
  double out[K];
  if (m_c == 1) {
    const double inv = (gram[0] > 0.0) ? 1.0 / sqrt(gram[0]) : 0.0;
#pragma unroll
    for (int c = 0; c < K; ++c) out[c] = s_C[0][c][slot] * inv;
  } else {
    // Gram-Schmidt of the m_c candidates in the Gram inner product, on
    // coefficient vectors (candidate a is e_a); rows r >= m_c stay unused
    double X[K][K];
#pragma unroll
    for (int r = 0; r < K; ++r)
#pragma unroll
      for (int a = 0; a < K; ++a) X[r][a] = (r == a && r < m_c) ? 1.0 : 0.0;
#pragma unroll
    for (int r = 0; r < K; ++r) {
      if (r < m_c) {
#pragma unroll
        for (int l = 0; l < K; ++l) {
          if (l < r) {
            const double g = quad<K>(gram, X[l], X[r]);
#pragma unroll
            for (int a = 0; a < K; ++a) X[r][a] -= g * X[l][a];
          }
        }
        const double nn = sqrt(fmax(quad<K>(gram, X[r], X[r]), 0.0));
        const double inv = (nn > 0.0) ? 1.0 / nn : 0.0;
#pragma unroll
        for (int a = 0; a < K; ++a) X[r][a] *= inv;
      }
    }
    // Rayleigh-Ritz: in candidate coordinates S acts as diag(theta), so
    // C^T (S Sigma S + S) C = Theta (Cc^T Sigma Cc) Theta + Theta
    double th[K];
#pragma unroll
    for (int a = 0; a < K; ++a) th[a] = s_th[a][slot];
    double Hc[Sym<K>::NS];
#pragma unroll
    for (int a = 0; a < K; ++a)
#pragma unroll
      for (int b = a; b < K; ++b) {
        double m = 0.0;
#pragma unroll
        for (int c = 0; c < K; ++c)
          m += s_C[a][c][slot] * (((w.sig_pos_mask >> c) & 1) ? 1.0 : -1.0) * s_C[b][c][slot];
        Hc[Sym<K>::at(a, b)] = th[a] * m * th[b] + ((a == b) ? th[a] : 0.0);
      }
    double H[Sym<K>::NS];
    double hscale = 0.0;
#pragma unroll
    for (int a = 0; a < K; ++a) hscale = fmax(hscale, fabs(th[a]));
#pragma unroll
    for (int r = 0; r < K; ++r)
#pragma unroll
      for (int q = r; q < K; ++q) {
        double acc = quad<K>(Hc, X[r], X[q]);
        if (r >= m_c || q >= m_c) acc = (r == q) ? 4.0 * hscale + 1.0 : 0.0;
        H[Sym<K>::at(r, q)] = acc;
      }
    double Y[K][K];
    jacobi_eig<K, true>(H, Y);
    // the Ritz vector of rank pos (ascending Ritz value)
    double z[K];
#pragma unroll
    for (int a = 0; a < K; ++a) z[a] = 0.0;
#pragma unroll
    for (int m = 0; m < K; ++m) {
      const double hm = H[Sym<K>::at(m, m)];
      int rk = 0;
#pragma unroll
      for (int m2 = 0; m2 < K; ++m2) {
        const double h2 = H[Sym<K>::at(m2, m2)];
        rk += (h2 < hm || (h2 == hm && m2 < m)) ? 1 : 0;
      }
      if (rk == pos) {
#pragma unroll
        for (int r = 0; r < K; ++r)
#pragma unroll
          for (int a = 0; a < K; ++a) z[a] += Y[r][m] * X[r][a];
      }
    }
#pragma unroll
    for (int c = 0; c < K; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int a = 0; a < K; ++a) acc += z[a] * s_C[a][c][slot];
      out[c] = acc;
    }
  }
#pragma unroll
  for (int c = 0; c < K; ++c) w.root_c[(size_t)i * K + c] = out[c];
  w.root_tv[i] = tau;
}


// ---------------------------------------------------------------------------
// Rank-2 location from residue signs (Sec. 2.2, Alg. 1a-1c; eq. (2)).
//
// alpha_s = -det [[0, u_s^T], [Sigma u_s, I + Sigma U^T D_s U]] with
// U^T D_s U = sum_{j != s} u_j u_j^T / (d_j - d_s) = -T_s, the same pole sweep as
// the pole counts.  An interval between consecutive poles holds an odd number
// of roots exactly when the residues at its ends have the same sign (virtual
// signs -1 below the first pole and +1 above the last), and the Courant-Weyl
// bounds leave two candidates for the number of roots below pole s, s - 1 + q
// and s + q (q = negative signs): the parity of the odd intervals up to s picks
// one.  This is the count Alg. 1a/1b/1c produce, formed by a prefix sum
// instead of a sequential scan.  Used only when every pole is simple and every
// residue is larger than a bound on its rounding error; otherwise the pole-count
// kernel runs.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void alpha_body(const Work& w, int bid) {
  constexpr int K = 2;
  constexpr int WV = Cfg<K>::WV, RPB = Cfg<K>::RPB, TP = Cfg<K>::TP, SPLIT = Cfg<K>::SPLIT;
  __shared__ double s_part[WV][6][RPB];
  __shared__ PoleTile<K, TP> s_tile[WV];
  if (update_cancelled(w.st)) return;
  const int n_s = w.info->n_s, n_d = w.info->n_d;
  if (n_s != n_d) {  // a multi-row pole: the residue formula does not apply
    if (bid == 0 && threadIdx.x == 0) atomicOr(&w.info->alpha_bad, 1);
    return;
  }
  const int s0 = bid * RPB;
  if (s0 >= n_s) return;
  const int lane = threadIdx.x & 63, slot = lane % RPB;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int s = min(s0 + slot, n_s - 1);
  const double d_s = w.rd[s];
  const int chunk = (n_d + WV - 1) / WV;
  const int jb = min(n_d, wv * chunk), je = min(n_d, jb + chunk);
  // T = sum u_j u_j^T / (d_s - d_j) and, for the error bound, sum |u_j u_j^T| / |d_s - d_j|
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  sweep_poles<K, TP, SPLIT>(w.rd, w.ru, jb, je, 0.0, d_s, s_tile[wv],
                            [&](double r, const double (&u)[K]) {
                              const double a = u[0] * r, b = u[1] * r;
                              acc[0] = fma(u[0], a, acc[0]);
                              acc[1] = fma(u[0], b, acc[1]);
                              acc[2] = fma(u[1], b, acc[2]);
                              acc[3] += fabs(u[0] * a);
                              acc[4] += fabs(u[0] * b);
                              acc[5] += fabs(u[1] * b);
                            });
  combine_parts<SPLIT>(acc);
  if (lane < RPB) {
#pragma unroll
    for (int e = 0; e < 6; ++e) s_part[wv][e][slot] = acc[e];
  }
  __syncthreads();
  if (wv != 0 || lane >= RPB || s0 + slot >= n_s) return;
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    double t = 0.0;
    for (int q = 0; q < WV; ++q) t += s_part[q][e][slot];
    acc[e] = t;
  }
  const double s1 = (w.sig_pos_mask & 1) ? 1.0 : -1.0, s2 = (w.sig_pos_mask & 2) ? 1.0 : -1.0;
  const double u1 = w.ru[(size_t)s * K], u2 = w.ru[(size_t)s * K + 1];
  // M = I - Sigma T (rows scaled by Sigma)
  const double m11 = 1.0 - s1 * acc[0], m12 = -s1 * acc[1];
  const double m21 = -s2 * acc[1], m22 = 1.0 - s2 * acc[2];
  const double alpha = u1 * (s1 * u1 * m22 - s2 * u2 * m12) - u2 * (s1 * u1 * m21 - s2 * u2 * m11);
  // rounding bound: the n-term sums and the 3 x 3 expansion
  const double a1 = fabs(u1), a2 = fabs(u2);
  const double bound = a1 * (a1 * (1.0 + acc[5]) + a2 * acc[4]) +
                       a2 * (a1 * acc[4] + a2 * (1.0 + acc[3]));
  const double tol = 4.0 * (double)(n_d + 8) * EPSU * bound;
  if (!(fabs(alpha) > tol)) atomicOr(&w.info->alpha_bad, 1);
  w.nu[s] = (alpha > 0.0) ? 1 : -1;
}

__global__ __launch_bounds__(64 * Cfg<2>::WV) void alpha_kernel(Work w) {
  alpha_body(w, blockIdx.x);
}

// Pole counts from the residue signs: one block; inclusive prefix count of the
// odd intervals, then the Courant-Weyl candidate with that parity.  Checks that
// the counts rise by 0, 1 or 2 per interval and end at n_d; otherwise leaves
// them to the pole-count kernel.
__global__ __launch_bounds__(LNT) void alpha_scan_kernel(Work w) {
  __shared__ int sh[LNT / 64 + 1];
  __shared__ int s_carry, s_bad, s_prev, s_prev_next;
  if (update_cancelled(w.st)) return;
  const int n_s = w.info->n_s, n_d = w.info->n_d;
  if (w.info->alpha_bad || n_s != n_d) return;
  const int q = w.info->q;
  if (threadIdx.x == 0) {
    s_carry = 0;
    s_bad = 0;
    s_prev = -1;  // virtual sign below the first pole
  }
  __syncthreads();
  // nu[] holds the residue signs on entry and the counts on exit; each chunk
  // reads all its signs before any of them is overwritten, and the sign of the
  // chunk's last pole is carried to the next chunk in s_prev
  for (int base = 0; base < n_s; base += LNT) {
    const int t = base + threadIdx.x;  // interval just below pole t
    const int last = min(base + LNT, n_s) - 1;
    int sg = 0, odd = 0;
    if (t < n_s) {
      sg = w.nu[t];
      const int left = (t == base) ? s_prev : w.nu[t - 1];
      odd = (left == sg) ? 1 : 0;
    }
    int tot = 0;
    const int excl = block_excl_scan<LNT>(odd, sh, &tot);  // synchronises the block
    const int incl = s_carry + excl + odd;                   // odd intervals among 0..t
    if (t == last) s_prev_next = sg;
    if (t < n_s) {
      const int lo = t - 1 + q;
      const int v = ((lo - incl) & 1) ? lo + 1 : lo;
      w.nu[t] = v;
      if (v < 0 || v > n_d) s_bad = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      s_carry += tot;
      s_prev = s_prev_next;
    }
    __syncthreads();
  }
  // the counts rise by 0, 1 or 2 per interval; the interval above the last pole
  // holds n_d - nu(last) roots, an odd number exactly when the last residue is
  // positive
  for (int t = threadIdx.x; t < n_s; t += LNT) {
    const int prev = (t == 0) ? 0 : w.nu[t - 1];
    const int d = w.nu[t] - prev;
    if (d < 0 || d > 2) s_bad = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int top = n_d - ((n_s > 0) ? w.nu[n_s - 1] : 0);
    if (top < 0 || top > 2 || ((top & 1) != (s_prev > 0 ? 1 : 0))) s_bad = 1;
    if (s_bad)
      w.info->alpha_bad = 1;
    else
      w.info->loc_alpha = 1;
  }
}

hipError_t launch_alpha_locate(const Work& w, hipStream_t s) {
  if (w.k != 2) return hipErrorInvalidValue;
  hipLaunchKernelGGL(alpha_kernel, dim3((w.n + Cfg<2>::RPB - 1) / Cfg<2>::RPB),
                     dim3(64 * Cfg<2>::WV), 0, s, w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(alpha_scan_kernel, dim3(1), dim3(LNT), 0, s, w);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Counts for a subset of the spectrum (Sec. 2.1: only the eigenvalues in an
// interval of interest; the first sub-problem, the count, decides which roots
// lie there).  For x = a and x = b: nu_red(x) = #{d_j < x} + neg(S(x)) - p over
// the reduced problem (S summed by the block, the inertia from its k x k
// eigenvalues), or the pole count when x is a pole; plus the number of deflated
// eigenvalues below x.  One block.
// ---------------------------------------------------------------------------
template <int K>
__global__ __launch_bounds__(256) void interval_count_kernel(Work w, double a, double b) {
  constexpr int NS = Sym<K>::NS;
  __shared__ double s_red[4][2 * NS];
  __shared__ int s_res[4];
  if (update_cancelled(w.st)) return;
  const int n_d = w.info->n_d, n_s = w.info->n_s, n_defl = w.info->n_defl;
  const double xs[2] = {a, b};
  double S[2][NS];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int e = 0; e < NS; ++e) S[q][e] = 0.0;
  for (int j = threadIdx.x; j < n_d; j += 256) {
    double u[K];
#pragma unroll
    for (int c = 0; c < K; ++c) u[c] = w.ru[(size_t)j * K + c];
    const double dj = w.rd[j];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const double r = recip(xs[q] - dj);
#pragma unroll
      for (int c1 = 0; c1 < K; ++c1)
#pragma unroll
        for (int c2 = c1; c2 < K; ++c2)
          S[q][Sym<K>::at(c1, c2)] = fma(u[c1] * r, u[c2], S[q][Sym<K>::at(c1, c2)]);
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int e = 0; e < NS; ++e) {
      const double t = wave_sum(S[q][e]);
      if (lane == 0) s_red[wv][q * NS + e] = t;
    }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int q = threadIdx.x;
    const double x = xs[q];
    int red;  // roots of the reduced problem below x
    if (!(x > -INFINITY)) {
      red = 0;
    } else if (!(x < INFINITY)) {
      red = n_d;
    } else {
      // segments strictly below x, and whether x is a pole
      int lo = 0, hi = n_s;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (w.rd[w.seg_start[mid]] < x)
          lo = mid + 1;
        else
          hi = mid;
      }
      if (lo < n_s && w.rd[w.seg_start[lo]] == x) {
        red = w.nu[lo];  // x is a pole: the pole count
      } else {
        double T[NS];
#pragma unroll
        for (int e = 0; e < NS; ++e)
          T[e] = s_red[0][q * NS + e] + s_red[1][q * NS + e] + s_red[2][q * NS + e] +
                 s_red[3][q * NS + e];
#pragma unroll
        for (int c = 0; c < K; ++c) T[Sym<K>::at(c, c)] -= ((w.sig_pos_mask >> c) & 1) ? 1.0 : -1.0;
        const int below = (lo < n_s) ? w.seg_start[lo] : n_d;  // rows with d_j < x
        red = below + neg_count<K>(T) - w.info->p;
      }
    }
    red = min(max(red, 0), n_d);
    // deflated eigenvalues strictly below x
    int lo = 0, hi = n_defl;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (w.dval[mid] < x)
        lo = mid + 1;
      else
        hi = mid;
    }
    s_res[2 * q] = red;
    s_res[2 * q + 1] = lo;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    w.info->r_lo = s_res[0];
    w.info->r_hi = max(s_res[0], s_res[2]);
    w.info->e_lo = s_res[1];
    w.info->e_hi = max(s_res[1], s_res[3]);
  }
}

template <int K>
static hipError_t interval_count_launch(const Work& w, double a, double b, hipStream_t s) {
  hipLaunchKernelGGL((interval_count_kernel<K>), dim3(1), dim3(256), 0, s, w, a, b);
  return hipGetLastError();
}

hipError_t launch_interval_count(const Work& w, double a, double b, hipStream_t s) {
  EIGUPD_SWITCH_K(w.k, interval_count_launch, w, a, b, s)
}

// ---------------------------------------------------------------------------
// Kernels: one instance (Work by value), a group of instances of one rank
// (Group), and the persistent root solver that takes (instance, root block)
// items from a queue.
// ---------------------------------------------------------------------------
template <int K>
__global__ __launch_bounds__(64 * Cfg<K>::WV) void polecount_kernel(Work w) {
  polecount_body<K>(w, blockIdx.x);
}
template <int K>
__global__ __launch_bounds__(64 * Cfg<K>::WV) void polecount_group(Group g) {
  const int i = group_instance(g, blockIdx.x);
  polecount_body<K>(g.works[i], blockIdx.x - g.prefix[i]);
}

__global__ __launch_bounds__(LNT) void locate_kernel(Work w) { locate_body(w); }
__global__ __launch_bounds__(LNT) void locate_group(const Work* __restrict__ works) {
  locate_body(works[blockIdx.x]);
}

template <int K>
__global__ __launch_bounds__(64 * RsCfg<K>::WV) void rootsolve_kernel(Work w) {
  rootsolve_body<K>(w);
}
template <int K>
__global__ __launch_bounds__(64 * RsCfg<K>::WV) void rootsolve_group(Group g) {
  rootsolve_body<K>(g.works[group_instance(g, blockIdx.x)]);
}
// A fixed grid of blocks; each takes the next item of the queue (an atomic
// counter that starts at 0) until all `total` items are taken.  Every block
// leaves the loop once the counter has passed `total`.
template <int K>
__global__ __launch_bounds__(64 * RsCfg<K>::WV) void rootsolve_persist(Group g, int total,
                                                                        int* queue) {
  __shared__ int s_item;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd(queue, 1);
    __syncthreads();
    const int item = s_item;
    if (item >= total) break;
    rootsolve_body<K>(g.works[group_instance(g, item)]);
  }
}

template <int K>
__global__ __launch_bounds__(64 * Cfg<K>::WV) void rootvec_kernel(Work w) {
  rootvec_body<K>(w, blockIdx.x);
}
template <int K>
__global__ __launch_bounds__(64 * Cfg<K>::WV) void rootvec_group(Group g) {
  const int i = group_instance(g, blockIdx.x);
  rootvec_body<K>(g.works[i], blockIdx.x - g.prefix[i]);
}

int root_blocks(int n) { return (n + 31) / 32; }
// Root-solver blocks the device holds at once (CUs x resident blocks per CU),
// looked up once per rank.
template <int K>
static int resident_solve_blocks_k() {
  static std::atomic<int> cached{0};
  int v = cached.load(std::memory_order_relaxed);
  if (v > 0) return v;
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per, reinterpret_cast<const void*>(&rootsolve_kernel<K>), 64 * RsCfg<K>::WV, 0) !=
          hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  v = max(cus * per, 1);
  cached.store(v, std::memory_order_relaxed);
  return v;
}
static int resident_solve_blocks(int k) {
  switch (k) {
    case 1: return resident_solve_blocks_k<1>();
    case 2: return resident_solve_blocks_k<2>();
    case 3: return resident_solve_blocks_k<3>();
    case 4: return resident_solve_blocks_k<4>();
    case 5: return resident_solve_blocks_k<5>();
    case 6: return resident_solve_blocks_k<6>();
    case 7: return resident_solve_blocks_k<7>();
    default: return resident_solve_blocks_k<8>();
  }
}

// Two roots per slot on average (a slot's refills balance the roots' differing
// iteration counts), but as many blocks as the device holds at once where that
// is more -- ranks whose solver fits several blocks per CU would otherwise
// leave CUs idle -- up to one root per slot.  The grid does not change the
// result of any root: every slot sums the same pole partition in the same order.
int solve_blocks(int n, int k) {
  const int two = (n + 2 * 8 - 1) / (2 * 8), one = (n + 8 - 1) / 8;
  return max(two, min(one, resident_solve_blocks(k)));
}

template <int K>
static hipError_t polecount_group_launch(const Group& g, int blocks, hipStream_t s) {
  static_assert(Cfg<K>::RPB == 32, "root_blocks assumes 32 roots per block");
  hipLaunchKernelGGL((polecount_group<K>), dim3(blocks), dim3(64 * Cfg<K>::WV), 0, s, g);
  return hipGetLastError();
}

template <int K>
static hipError_t rootsolve_group_launch(const Group& gs, int solve_blocks, const Group& gv,
                                         int vec_blocks, int persistent_grid, int* queue,
                                         hipStream_t s) {
  hipError_t e;
  bool persistent = false;
  // ranks >= 7: the persistent loop around the solver does not fit its
  // registers; the grouped launch computes the same numbers
  if constexpr (K <= 6) {
    if (persistent_grid > 0) {
      hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, s, queue, 1);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((rootsolve_persist<K>), dim3(min(persistent_grid, solve_blocks)),
                         dim3(64 * RsCfg<K>::WV), 0, s, gs, solve_blocks, queue);
      persistent = true;
    }
  }
  if (!persistent)
    hipLaunchKernelGGL((rootsolve_group<K>), dim3(solve_blocks), dim3(64 * RsCfg<K>::WV), 0, s,
                       gs);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((rootvec_group<K>), dim3(vec_blocks), dim3(64 * Cfg<K>::WV), 0, s, gv);
  return hipGetLastError();
}

hipError_t launch_polecount_group(int k, const Group& g, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  EIGUPD_SWITCH_K(k, polecount_group_launch, g, blocks, s)
}

hipError_t launch_locate_group(const Work* works, int ninst, hipStream_t s) {
  if (ninst <= 0) return hipSuccess;
  hipLaunchKernelGGL(locate_group, dim3(ninst), dim3(LNT), 0, s, works);
  return hipGetLastError();
}

hipError_t launch_rootsolve_group(int k, const Group& gs, int solve_blocks, const Group& gv,
                                  int vec_blocks, int persistent_grid, int* queue,
                                  hipStream_t s) {
  if (solve_blocks <= 0) return hipSuccess;
  EIGUPD_SWITCH_K(k, rootsolve_group_launch, gs, solve_blocks, gv, vec_blocks, persistent_grid,
                  queue, s)
}

template <int K>
static hipError_t polecount_launch(const Work& w, hipStream_t s) {
  const int grid = (w.n + Cfg<K>::RPB - 1) / Cfg<K>::RPB;
  hipLaunchKernelGGL((polecount_kernel<K>), dim3(grid), dim3(64 * Cfg<K>::WV), 0, s, w);
  return hipGetLastError();
}

template <int K>
static hipError_t rootsolve_launch(const Work& w, int nroots, hipStream_t s) {
  if (nroots <= 0) return hipSuccess;
  static_assert(RsCfg<K>::RPB == 8, "solve_blocks assumes 8 slots per block");
  hipLaunchKernelGGL((rootsolve_kernel<K>), dim3(solve_blocks(nroots, K)), dim3(64 * RsCfg<K>::WV),
                     0, s, w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int grid = (nroots + Cfg<K>::RPB - 1) / Cfg<K>::RPB;
  hipLaunchKernelGGL((rootvec_kernel<K>), dim3(grid), dim3(64 * Cfg<K>::WV), 0, s, w);
  return hipGetLastError();
}

#define EIGUPD_DISPATCH_K(fn)                 \
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

hipError_t launch_polecount(const Work& w, hipStream_t s) { EIGUPD_DISPATCH_K(polecount_launch) }

hipError_t launch_rootsolve(const Work& w, hipStream_t s, int nroots) {
  EIGUPD_SWITCH_K(w.k, rootsolve_launch, w, nroots < 0 ? w.n : nroots, s)
}

hipError_t launch_locate(const Work& w, hipStream_t s) {
  hipLaunchKernelGGL(locate_kernel, dim3(1), dim3(LNT), 0, s, w);
  return hipGetLastError();
}

}  // namespace eigupd
