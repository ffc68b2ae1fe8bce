/*
 * eigref.c -- plain, slow FP64 CPU oracle for the rank-k symmetric eigen-update
 * of Oh & Hu, "Multiple-rank Modification of Symmetric Eigenvalue Problem"
 * (arXiv:1706.00773).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU product path
 * never links, loads or calls it, and the two share no code.
 *
 * Problem (Sec. 2.1): A = Q diag(lam) Q^T is known, the perturbation is
 * K Sigma K^T with K n-by-k and Sigma = diag(sigma_c), sigma_c = +-1 (the paper
 * writes K K^T; the one-column-one-row update of Sec. 2.2, Step 2, needs one
 * negative sign).  With U = Q^T K (Sec. 2.1, below eq. (1)) the new
 * eigenvalues are the eigenvalues of D + U Sigma U^T, D = diag(lam), and the
 * new eigenvectors are Q w with w the eigenvectors of that matrix (Sec. 2.4).
 *
 * Every quantity is computed in the most direct way:
 *   - U by plain dot products;
 *   - the count nu(x) = #{eigenvalues of D + U Sigma U^T strictly below x}
 *     from the inertia of the bordered matrix [[D - xI, U], [U^T, -Sigma]]
 *     (Haynsworth): nu(x) = #{lam_j < x} + neg(S(x)) - p with
 *     S(x) = sum_j u_j u_j^T / (x - lam_j) - Sigma and p = #{sigma_c = +1}.
 *     This is the integer that the paper's modified Sturm chain produces
 *     (Sec. 2.2, sign changes of the chain at a and b); neg() comes from a
 *     plain cyclic Jacobi eigensolve of the k-by-k matrix;
 *   - each eigenvalue by bisection on that count inside its Courant-Weyl
 *     window (Sec. 2.2) -- the paper's divide-and-conquer zero finder
 *     (Sec. 2.3) with one interior point per step, driven by the count;
 *   - each eigenvector from Sec. 2.4, eq. (10): w = (lam' I - D)^{-1} U c,
 *     c a null vector of the k-by-k matrix S(lam'), normalised;
 *   - Q' = Q W by a plain blocked triple loop.
 *
 * Readings of the paper taken here (each is also listed in the design notes):
 *   - The sign of eq. (2): f(x) = det(I - Sigma U^T (xI - D)^{-1} U)
 *     = 1 + sum_i alpha_i / (lam_i - x) with
 *     alpha_i = -det [[0, u_i^T], [Sigma u_i, I + Sigma U^T D_i U]];
 *     for k = 1 this is sigma u_i^2, the rank-1 secular function of Sec. 1.
 *   - The only deflation done here is of rows of U that are exactly zero
 *     (their eigenpair is (lam_j, e_j)).
 *   - Eigenvalues are returned ascending; each eigenvector's largest-magnitude
 *     entry in the Q basis is made positive (ties: lowest index).
 *
 * Shifted coordinates: a point is held as x = lam[o] + tau, and every
 * difference x - lam_j is formed as tau - (lam_j - lam_o), so that the
 * distance to the origin pole o is exact.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define REF_OK 0
#define REF_EINVAL -1
#define REF_ENOMEM -2
#define REF_EPOLE -3

static const double EPS = DBL_EPSILON / 2.0; /* unit round-off 2^-53 */

/* ------------------------------------------------------------------------ */
/* Threads                                                                   */
/* ------------------------------------------------------------------------ */
void eigref_set_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

int eigref_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Small dense helpers                                                        */
/* ------------------------------------------------------------------------ */

/* Cyclic Jacobi eigensolver for a symmetric m-by-m matrix a (row-major,
 * destroyed).  Eigenvalues ascending in w; if V is not NULL, V[r*m + c] is
 * component r of the unit eigenvector for w[c].  Textbook method (two-sided
 * plane rotations chosen to annihilate a_pq, Golub & Van Loan, Sec. 8.5). */
static void jacobi_sym(int m, double *a, double *w, double *V) {
  if (V) {
    for (int r = 0; r < m; ++r)
      for (int c = 0; c < m; ++c) V[r * m + c] = (r == c) ? 1.0 : 0.0;
  }
  /* Stop at a negligible off-diagonal, or once a sweep no longer reduces it:
   * then the rotations only stir rounding errors (the off-diagonal has reached
   * its floor, about eps ||a||), and further sweeps change nothing that
   * matters. */
  double off_prev = INFINITY;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int r = 0; r < m; ++r)
      for (int c = 0; c < m; ++c) {
        double v = a[r * m + c] * a[r * m + c];
        tot += v;
        if (r != c) off += v;
      }
    if (off == 0.0 || off <= 1e-36 * tot || !(off < off_prev)) break;
    off_prev = off;
    for (int p = 0; p < m - 1; ++p)
      for (int q = p + 1; q < m; ++q) {
        double apq = a[p * m + q];
        if (apq == 0.0) continue;
        double app = a[p * m + p], aqq = a[q * m + q];
        double theta = (aqq - app) / (2.0 * apq);
        double t;
        if (fabs(theta) > 1e150)
          t = 0.5 / theta;
        else
          t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < m; ++r) { /* columns p, q */
          double arp = a[r * m + p], arq = a[r * m + q];
          a[r * m + p] = c * arp - s * arq;
          a[r * m + q] = s * arp + c * arq;
        }
        for (int r = 0; r < m; ++r) { /* rows p, q */
          double apr = a[p * m + r], aqr = a[q * m + r];
          a[p * m + r] = c * apr - s * aqr;
          a[q * m + r] = s * apr + c * aqr;
        }
        if (V)
          for (int r = 0; r < m; ++r) {
            double vrp = V[r * m + p], vrq = V[r * m + q];
            V[r * m + p] = c * vrp - s * vrq;
            V[r * m + q] = s * vrp + c * vrq;
          }
      }
  }
  for (int i = 0; i < m; ++i) w[i] = a[i * m + i];
  /* selection sort ascending, carrying the eigenvector columns */
  for (int i = 0; i < m; ++i) {
    int b = i;
    for (int j = i + 1; j < m; ++j)
      if (w[j] < w[b]) b = j;
    if (b != i) {
      double tw = w[i];
      w[i] = w[b];
      w[b] = tw;
      if (V)
        for (int r = 0; r < m; ++r) {
          double tv = V[r * m + i];
          V[r * m + i] = V[r * m + b];
          V[r * m + b] = tv;
        }
    }
  }
}

/* Determinant by Gaussian elimination with partial pivoting (a destroyed). */
static double det_gepp(int m, double *a) {
  double det = 1.0;
  for (int c = 0; c < m; ++c) {
    int piv = c;
    for (int r = c + 1; r < m; ++r)
      if (fabs(a[r * m + c]) > fabs(a[piv * m + c])) piv = r;
    if (a[piv * m + c] == 0.0) return 0.0;
    if (piv != c) {
      for (int j = 0; j < m; ++j) {
        double t = a[c * m + j];
        a[c * m + j] = a[piv * m + j];
        a[piv * m + j] = t;
      }
      det = -det;
    }
    det *= a[c * m + c];
    for (int r = c + 1; r < m; ++r) {
      double f = a[r * m + c] / a[c * m + c];
      for (int j = c; j < m; ++j) a[r * m + j] -= f * a[c * m + j];
    }
  }
  return det;
}

static int n_positive_sigma(int64_t k, const int8_t *sigma) {
  int p = 0;
  for (int64_t c = 0; c < k; ++c) p += (sigma[c] > 0);
  return p;
}

static int check_common(int64_t n, int64_t k, const double *lam, const double *U,
                        const int8_t *sigma) {
  if (n < 1 || k < 1 || k > 64 || !lam || !U || !sigma) return REF_EINVAL;
  for (int64_t c = 0; c < k; ++c)
    if (sigma[c] != 1 && sigma[c] != -1) return REF_EINVAL;
  for (int64_t j = 1; j < n; ++j)
    if (!(lam[j] >= lam[j - 1])) return REF_EINVAL;
  return REF_OK;
}

static int row_is_zero(int64_t k, const double *u) {
  for (int64_t c = 0; c < k; ++c)
    if (u[c] != 0.0) return 0;
  return 1;
}

/* ------------------------------------------------------------------------ */
/* U = Q^T K   (Sec. 2.1; Sec. 2.4 calls it L)                                */
/* Q is n-by-n column-major (leading dimension ldq), K n-by-k column-major   */
/* (ldk).  U is written row-major: U[j*k + c] = column j of Q dot column c.  */
/* ------------------------------------------------------------------------ */
int eigref_qtk(int64_t n, int64_t k, const double *Q, int64_t ldq, const double *K,
               int64_t ldk, double *U) {
  if (n < 1 || k < 1 || ldq < n || ldk < n || !Q || !K || !U) return REF_EINVAL;
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; ++j)
    for (int64_t c = 0; c < k; ++c) {
      double s = 0.0;
      for (int64_t r = 0; r < n; ++r) s += Q[r + j * ldq] * K[r + c * ldk];
      U[j * k + c] = s;
    }
  return REF_OK;
}

/* ------------------------------------------------------------------------ */
/* The count nu(x) (modified Sturm count, Sec. 2.2).                         */
/* x = lam[origin] + tau, or x = tau when origin < 0.  Rows of U that are    */
/* zero add nothing to S(x) but are counted by #{lam_j < x}.  Returns -1 if  */
/* x is a pole (x == lam_j for a row with u_j != 0).                         */
/* ------------------------------------------------------------------------ */
static int64_t count_below(int64_t n, int64_t k, const double *lam, const double *U,
                           const int8_t *sigma, int64_t origin, double tau, double *S,
                           double *w) {
  for (int64_t a = 0; a < k * k; ++a) S[a] = 0.0;
  int64_t below = 0;
  for (int64_t j = 0; j < n; ++j) {
    double y = (origin >= 0) ? tau - (lam[j] - lam[origin]) : tau - lam[j]; /* x - lam_j */
    if (y > 0.0) ++below;
    const double *u = U + j * k;
    if (row_is_zero(k, u)) continue;
    if (y == 0.0) return -1;
    for (int64_t a = 0; a < k; ++a)
      for (int64_t b = 0; b < k; ++b) S[a * k + b] += u[a] * u[b] / y;
  }
  for (int64_t c = 0; c < k; ++c) S[c * k + c] -= (double)sigma[c];
  jacobi_sym((int)k, S, w, NULL);
  int64_t neg = 0;
  for (int64_t c = 0; c < k; ++c) neg += (w[c] < 0.0);
  return below + neg - n_positive_sigma(k, sigma);
}

int64_t eigref_count(int64_t n, int64_t k, const double *lam, const double *U,
                     const int8_t *sigma, int64_t origin, double tau) {
  if (check_common(n, k, lam, U, sigma) != REF_OK || origin >= n) return -2;
  double *S = (double *)malloc(sizeof(double) * (size_t)(k * k + k));
  if (!S) return -2;
  int64_t r = count_below(n, k, lam, U, sigma, origin, tau, S, S + k * k);
  free(S);
  return r;
}

/* nu(lam_j): the count exactly at a pole whose row is nonzero, from the
 * bordered (k+1)-by-(k+1) matrix B_j = [[0, u_j^T], [u_j, T_j]],
 * T_j = sum_{l: lam_l != lam_j} u_l u_l^T / (lam_j - lam_l) - Sigma:
 *   nu(lam_j) = #{lam_l < lam_j} + neg(B_j) - p.
 * Requires every other row with lam_l == lam_j to be zero. */
static int64_t pole_count_at(int64_t n, int64_t k, const double *lam, const double *U,
                             const int8_t *sigma, int64_t j, double *B /* (k+1)^2 + k+1 */) {
  int64_t m = k + 1;
  for (int64_t a = 0; a < m * m; ++a) B[a] = 0.0;
  int64_t below = 0;
  for (int64_t l = 0; l < n; ++l) {
    if (lam[l] < lam[j]) ++below;
    if (lam[l] == lam[j]) {
      if (l != j && !row_is_zero(k, U + l * k)) return -2;
      continue;
    }
    double y = lam[j] - lam[l];
    const double *u = U + l * k;
    for (int64_t a = 0; a < k; ++a)
      for (int64_t b = 0; b < k; ++b) B[(a + 1) * m + (b + 1)] += u[a] * u[b] / y;
  }
  for (int64_t c = 0; c < k; ++c) {
    B[(c + 1) * m + (c + 1)] -= (double)sigma[c];
    B[0 * m + (c + 1)] = U[j * k + c];
    B[(c + 1) * m + 0] = U[j * k + c];
  }
  jacobi_sym((int)m, B, B + m * m, NULL);
  int64_t neg = 0;
  for (int64_t c = 0; c < m; ++c) neg += (B[m * m + c] < 0.0);
  return below + neg - n_positive_sigma(k, sigma);
}

int64_t eigref_pole_count(int64_t n, int64_t k, const double *lam, const double *U,
                          const int8_t *sigma, int64_t j) {
  if (check_common(n, k, lam, U, sigma) != REF_OK || j < 0 || j >= n) return -2;
  if (row_is_zero(k, U + j * k)) return -2;
  int64_t m = k + 1;
  double *B = (double *)calloc((size_t)(m * m + m), sizeof(double));
  if (!B) return -2;
  int64_t r = pole_count_at(n, k, lam, U, sigma, j, B);
  free(B);
  return r;
}

/* ------------------------------------------------------------------------ */
/* Secular function f(x) = det(I_k - Sigma U^T (xI - D)^{-1} U)   (eq. (1)) */
/* ------------------------------------------------------------------------ */
int eigref_secular_det(int64_t n, int64_t k, const double *lam, const double *U,
                       const int8_t *sigma, double x, double *f) {
  if (check_common(n, k, lam, U, sigma) != REF_OK || !f) return REF_EINVAL;
  double *M = (double *)calloc((size_t)(k * k), sizeof(double));
  if (!M) return REF_ENOMEM;
  for (int64_t j = 0; j < n; ++j) {
    const double *u = U + j * k;
    if (row_is_zero(k, u)) continue;
    double y = x - lam[j];
    if (y == 0.0) {
      free(M);
      return REF_EPOLE;
    }
    for (int64_t a = 0; a < k; ++a)
      for (int64_t b = 0; b < k; ++b) M[a * k + b] += u[a] * u[b] / y;
  }
  /* I - Sigma M : row a scaled by sigma_a */
  for (int64_t a = 0; a < k; ++a)
    for (int64_t b = 0; b < k; ++b) M[a * k + b] = (a == b ? 1.0 : 0.0) - sigma[a] * M[a * k + b];
  *f = det_gepp((int)k, M);
  free(M);
  return REF_OK;
}

/* alpha_i, the residue coefficient of the multiple-rank secular function
 * (eq. (2), eq. (3)), read as
 *   alpha_i = -det [[0, u_i^T], [Sigma u_i, I + Sigma U^T D_i U]],
 * D_i = diag(1/(lam_j - lam_i)) with 0 in position i, so that
 * f(x) = 1 + sum_i alpha_i / (lam_i - x).  Poles must be distinct. */
int eigref_alpha(int64_t n, int64_t k, const double *lam, const double *U,
                 const int8_t *sigma, int64_t i, double *alpha) {
  if (check_common(n, k, lam, U, sigma) != REF_OK || i < 0 || i >= n || !alpha)
    return REF_EINVAL;
  int64_t m = k + 1;
  double *B = (double *)calloc((size_t)(m * m), sizeof(double));
  if (!B) return REF_ENOMEM;
  /* G = U^T D_i U */
  for (int64_t j = 0; j < n; ++j) {
    if (j == i) continue;
    if (lam[j] == lam[i]) {
      free(B);
      return REF_EPOLE;
    }
    double dj = 1.0 / (lam[j] - lam[i]);
    const double *u = U + j * k;
    for (int64_t a = 0; a < k; ++a)
      for (int64_t b = 0; b < k; ++b) B[(a + 1) * m + (b + 1)] += u[a] * u[b] * dj;
  }
  for (int64_t a = 0; a < k; ++a) {
    for (int64_t b = 0; b < k; ++b) B[(a + 1) * m + (b + 1)] *= sigma[a];
    B[(a + 1) * m + (a + 1)] += 1.0;
    B[0 * m + (a + 1)] = U[i * k + a];
    B[(a + 1) * m + 0] = sigma[a] * U[i * k + a];
  }
  *alpha = -det_gepp((int)m, B);
  free(B);
  return REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Brute force: cyclic Jacobi on an explicit symmetric m-by-m matrix.        */
/* A column-major (symmetric, so either order); w ascending; V column-major  */
/* m-by-m (column c = eigenvector of w[c]) or NULL.                          */
/* ------------------------------------------------------------------------ */
int eigref_jacobi(int64_t m, const double *A, double *w, double *V) {
  if (m < 1 || m > 4096 || !A || !w) return REF_EINVAL;
  double *a = (double *)malloc(sizeof(double) * (size_t)(m * m));
  double *Vr = V ? (double *)malloc(sizeof(double) * (size_t)(m * m)) : NULL;
  if (!a || (V && !Vr)) {
    free(a);
    free(Vr);
    return REF_ENOMEM;
  }
  for (int64_t r = 0; r < m; ++r)
    for (int64_t c = 0; c < m; ++c) a[r * m + c] = A[r + c * m];
  jacobi_sym((int)m, a, w, Vr);
  if (V)
    for (int64_t r = 0; r < m; ++r)
      for (int64_t c = 0; c < m; ++c) V[r + c * m] = Vr[r * m + c];
  free(a);
  free(Vr);
  return REF_OK;
}

/* ------------------------------------------------------------------------ */
/* One eigenvalue by bisection on the count (Sec. 2.2 location, Sec. 2.3    */
/* zero finder with one interior point per step).                           */
/* ------------------------------------------------------------------------ */

/* Smallest index t with lam[t] > v among rows with nonzero u (the "active"
 * poles); act[] lists their indices ascending. Returns na if none. */
static int64_t first_active_above(int64_t na, const int64_t *act, const double *lam, double v) {
  int64_t lo = 0, hi = na;
  while (lo < hi) {
    int64_t mid = (lo + hi) / 2;
    if (lam[act[mid]] > v)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

static int is_active_pole(int64_t na, const int64_t *act, const double *lam, double v) {
  int64_t t = first_active_above(na, act, lam, v);
  return (t > 0 && lam[act[t - 1]] == v);
}

typedef struct {
  int64_t n, k;
  const double *lam;
  const double *U;
  const int8_t *sigma;
  int p, q;
  int64_t na;         /* number of active (nonzero-row) poles */
  const int64_t *act; /* their indices */
  double lower, upper; /* outer bounds on all eigenvalues */
} problem_t;

/* eigenvalue index i (0-based over all n eigenvalues): returns x = lam[*o] + *tau
 * (or x = *tau when *o < 0) and the number of count evaluations. */
/* The bracket (lo, hi) has converged in absolute terms but an active pole lies
 * strictly inside it: the root is within rounding of that pole.  If that pole
 * value is unique among the active rows, decide the side of the root with the
 * count at the pole and continue in coordinates centred on it (so that the
 * distance to that pole, which eq. (10) divides by, is resolved to full
 * relative precision).  Returns the pole index, or -1 (keep the absolute
 * answer). */
static int64_t onto_pole(const problem_t *P, int64_t target, double lo, double hi, double *tlo,
                         double *thi, double *B) {
  int64_t t = first_active_above(P->na, P->act, P->lam, lo);
  if (t >= P->na || !(P->lam[P->act[t]] < hi)) return -1;
  int64_t p = P->act[t];
  if (t + 1 < P->na && P->lam[P->act[t + 1]] < hi) return -1; /* two poles inside */
  int64_t c = pole_count_at(P->n, P->k, P->lam, P->U, P->sigma, p, B);
  if (c < 0) return -1;
  if (c >= target) { /* the root lies below the pole */
    *tlo = lo - P->lam[p];
    *thi = 0.0;
  } else {
    *tlo = 0.0;
    *thi = hi - P->lam[p];
  }
  return p;
}

static int solve_one(const problem_t *P, int64_t i, int64_t *o_out, double *tau_out,
                     double *val_out, double *S, double *w) {
  const int64_t n = P->n, k = P->k;
  const double *lam = P->lam;
  const int64_t target = i + 1; /* 1-based: need nu(x) >= target <=> x > lam'_i */
  /* Courant-Weyl window (Sec. 2.2): lam_{i-q} <= lam'_i <= lam_{i+p} */
  double lo = (i - P->q >= 0) ? lam[i - P->q] : P->lower;
  double hi = (i + P->p <= n - 1) ? lam[i + P->p] : P->upper;
  int evals = 0;
  int64_t o = -1;
  double tlo = 0.0, thi = 0.0;
  /* phase 1: absolute coordinates until no active pole lies strictly inside */
  for (;;) {
    int64_t t = first_active_above(P->na, P->act, lam, lo);
    int inside = (t < P->na && lam[P->act[t]] < hi);
    if (!inside) break;
    double mid = lo + (hi - lo) / 2.0;
    if (is_active_pole(P->na, P->act, lam, mid)) mid = nextafter(mid, hi);
    if (hi - lo <= 2.0 * EPS * fmax(fabs(lo), fabs(hi)) || !(mid > lo && mid < hi) ||
        is_active_pole(P->na, P->act, lam, mid)) {
      o = onto_pole(P, target, lo, hi, &tlo, &thi, S);
      if (o >= 0) goto shifted;
      *o_out = -1;
      *tau_out = lo + (hi - lo) / 2.0;
      *val_out = *tau_out;
      return evals;
    }
    int64_t c = count_below(n, k, lam, P->U, P->sigma, -1, mid, S, w);
    ++evals;
    if (c >= target)
      hi = mid;
    else
      lo = mid;
  }
  /* the bracket lies between two adjacent active poles a <= lo < hi <= b */
  int64_t t = first_active_above(P->na, P->act, lam, lo);
  int64_t ia = (t > 0) ? P->act[t - 1] : -1; /* pole at or below lo */
  int64_t ib = (t < P->na) ? P->act[t] : -1;  /* pole at or above hi */
  if (ia >= 0 && lam[ia] > lo) ia = -1;
  if (ia >= 0 && ib >= 0) {
    double a = lam[ia], b = lam[ib];
    double m = a + (b - a) / 2.0;
    if (lo >= m)
      o = ib;
    else if (hi <= m)
      o = ia;
    else {
      if (is_active_pole(P->na, P->act, lam, m)) m = nextafter(m, b);
      int64_t c = count_below(n, k, lam, P->U, P->sigma, -1, m, S, w);
      ++evals;
      if (c >= target) {
        hi = m;
        o = ia;
      } else {
        lo = m;
        o = ib;
      }
    }
  } else if (ia >= 0) {
    o = ia;
  } else if (ib >= 0) {
    o = ib;
  } else {
    o = -1; /* no active pole at all: every row of U is zero */
  }
  if (o < 0) {
    /* U == 0: the count only sees lam; plain bisection in x */
    while (hi - lo > 2.0 * EPS * fmax(fabs(lo), fabs(hi))) {
      double mid = lo + (hi - lo) / 2.0;
      if (!(mid > lo && mid < hi)) break;
      int64_t c = count_below(n, k, lam, P->U, P->sigma, -1, mid, S, w);
      ++evals;
      if (c >= target)
        hi = mid;
      else
        lo = mid;
    }
    *o_out = -1;
    *tau_out = lo + (hi - lo) / 2.0;
    *val_out = *tau_out;
    return evals;
  }
  /* phase 2: bisection in shifted coordinates tau = x - lam[o] */
  tlo = lo - lam[o];
  thi = hi - lam[o];
shifted:
  for (;;) {
    if (thi - tlo <= 2.0 * EPS * fmax(fabs(tlo), fabs(thi))) break;
    double tm = tlo + (thi - tlo) / 2.0;
    if (!(tm > tlo && tm < thi)) break;
    int64_t c = count_below(n, k, lam, P->U, P->sigma, o, tm, S, w);
    ++evals;
    if (c < 0) break; /* cannot happen: tm != 0 inside one pole interval */
    if (c >= target)
      thi = tm;
    else
      tlo = tm;
  }
  *o_out = o;
  *tau_out = tlo + (thi - tlo) / 2.0;
  *val_out = lam[o] + *tau_out;
  return evals;
}

static int setup_problem(problem_t *P, int64_t n, int64_t k, const double *lam,
                         const double *U, const int8_t *sigma, int64_t **act_store) {
  P->n = n;
  P->k = k;
  P->lam = lam;
  P->U = U;
  P->sigma = sigma;
  P->p = n_positive_sigma(k, sigma);
  P->q = (int)k - P->p;
  int64_t *act = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  if (!act) return REF_ENOMEM;
  int64_t na = 0;
  for (int64_t j = 0; j < n; ++j)
    if (!row_is_zero(k, U + j * k)) act[na++] = j;
  P->na = na;
  P->act = act;
  *act_store = act;
  /* outer bounds (Weyl): lam_1 - sum_{sigma<0} ||U_c||^2 <= lam' <= lam_n + sum_{sigma>0} ||U_c||^2 */
  double neg = 0.0, pos = 0.0, amax = 0.0;
  for (int64_t c = 0; c < k; ++c) {
    double s = 0.0;
    for (int64_t j = 0; j < n; ++j) s += U[j * k + c] * U[j * k + c];
    if (sigma[c] < 0)
      neg += s;
    else
      pos += s;
  }
  for (int64_t j = 0; j < n; ++j) amax = fmax(amax, fabs(lam[j]));
  double pad = 16.0 * EPS * (amax + neg + pos) + DBL_MIN;
  P->lower = lam[0] - neg * (1.0 + 1e-10) - pad;
  P->upper = lam[n - 1] + pos * (1.0 + 1e-10) + pad;
  return REF_OK;
}

/* Eigenvalues with the given 0-based indices (idx == NULL: all n).
 * out_val[t] = lam'_{idx[t]}; out_origin/out_tau (optional) give the shifted
 * representation; out_evals (optional) the number of count evaluations. */
int eigref_eigvals(int64_t n, int64_t k, const double *lam, const double *U,
                   const int8_t *sigma, int64_t nidx, const int64_t *idx, double *out_val,
                   int64_t *out_origin, double *out_tau, int32_t *out_evals) {
  if (check_common(n, k, lam, U, sigma) != REF_OK || !out_val) return REF_EINVAL;
  if (!idx) nidx = n;
  for (int64_t t = 0; t < nidx; ++t)
    if (idx && (idx[t] < 0 || idx[t] >= n)) return REF_EINVAL;
  problem_t P;
  int64_t *act = NULL;
  if (setup_problem(&P, n, k, lam, U, sigma, &act) != REF_OK) return REF_ENOMEM;
  int err = REF_OK;
#pragma omp parallel
  {
    double *S = (double *)malloc(sizeof(double) * (size_t)((k + 1) * (k + 1) + (k + 1)));
    if (!S) {
#pragma omp atomic write
      err = REF_ENOMEM;
    }
#pragma omp for schedule(dynamic, 4)
    for (int64_t t = 0; t < nidx; ++t) {
      if (!S) continue;
      int64_t i = idx ? idx[t] : t;
      int64_t o;
      double tau, val;
      int ev = solve_one(&P, i, &o, &tau, &val, S, S + k * k);
      out_val[t] = val;
      if (out_origin) out_origin[t] = o;
      if (out_tau) out_tau[t] = tau;
      if (out_evals) out_evals[t] = ev;
    }
    free(S);
  }
  free(act);
  return err;
}

/* ------------------------------------------------------------------------ */
/* Eigenvectors in the Q basis (Sec. 2.4, eq. (10)).                          */
/* For each root (origin[t], tau[t]) the k-by-k matrix S(lam') is formed in   */
/* shifted coordinates, c is the eigenvector of its smallest-magnitude        */
/* eigenvalue, w_j = u_j^T c / (lam' - lam_j) for nonzero rows and 0 for zero */
/* rows, then w is normalised and signed.  A run of nmult roots that share   */
/* one value (cluster[t] = position of root t inside its run, mult[t] = run  */
/* length) takes the nmult smallest-magnitude eigenvectors, orthonormalised   */
/* in the inner product <c, c'> = c^T (U^T (lam' I - D)^{-2} U) c' (which     */
/* makes the resulting w mutually orthonormal), and picks number cluster[t].  */
/* cluster/mult may be NULL (all simple).  W is n-by-nvec column-major.       */
/* ------------------------------------------------------------------------ */
static void sign_and_store(int64_t n, double *w) {
  int64_t b = 0;
  for (int64_t j = 1; j < n; ++j)
    if (fabs(w[j]) > fabs(w[b])) b = j;
  if (w[b] < 0.0)
    for (int64_t j = 0; j < n; ++j) w[j] = -w[j];
}

static void one_vector(int64_t n, int64_t k, const double *lam, const double *U,
                       const int8_t *sigma, int64_t o, double tau, int64_t pos, int64_t mult,
                       double *S, double *G, double *th, double *V, double *w) {
  /* S(x) and G(x) = sum_j u_j u_j^T / (x - lam_j)^2 */
  for (int64_t a = 0; a < k * k; ++a) {
    S[a] = 0.0;
    G[a] = 0.0;
  }
  for (int64_t j = 0; j < n; ++j) {
    const double *u = U + j * k;
    if (row_is_zero(k, u)) continue;
    double y = (o >= 0) ? tau - (lam[j] - lam[o]) : tau - lam[j];
    for (int64_t a = 0; a < k; ++a)
      for (int64_t b = 0; b < k; ++b) {
        S[a * k + b] += u[a] * u[b] / y;
        G[a * k + b] += u[a] * u[b] / (y * y);
      }
  }
  for (int64_t c = 0; c < k; ++c) S[c * k + c] -= (double)sigma[c];
  jacobi_sym((int)k, S, th, V);
  /* order eigenvector indices by |theta| ascending */
  int64_t ord[64];
  for (int64_t c = 0; c < k; ++c) ord[c] = c;
  for (int64_t a = 0; a < k; ++a)
    for (int64_t b = a + 1; b < k; ++b)
      if (fabs(th[ord[b]]) < fabs(th[ord[a]])) {
        int64_t t = ord[a];
        ord[a] = ord[b];
        ord[b] = t;
      }
  if (mult < 1) mult = 1;
  if (mult > k) mult = k;
  if (pos >= mult) pos = mult - 1;
  /* Gram-Schmidt of the mult chosen vectors in the G inner product */
  double C[64 * 64];
  for (int64_t m = 0; m < mult; ++m)
    for (int64_t a = 0; a < k; ++a) C[m * k + a] = V[a * k + ord[m]];
  for (int64_t m = 0; m <= pos; ++m) {
    double *cm = C + m * k;
    for (int64_t l = 0; l < m; ++l) {
      double *cl = C + l * k, g = 0.0;
      for (int64_t a = 0; a < k; ++a)
        for (int64_t b = 0; b < k; ++b) g += cl[a] * G[a * k + b] * cm[b];
      for (int64_t a = 0; a < k; ++a) cm[a] -= g * cl[a];
    }
    double nn = 0.0;
    for (int64_t a = 0; a < k; ++a)
      for (int64_t b = 0; b < k; ++b) nn += cm[a] * G[a * k + b] * cm[b];
    nn = sqrt(nn);
    if (nn > 0.0)
      for (int64_t a = 0; a < k; ++a) cm[a] /= nn;
  }
  const double *c = C + pos * k;
  double nrm = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    const double *u = U + j * k;
    if (row_is_zero(k, u)) {
      w[j] = 0.0;
      continue;
    }
    double y = (o >= 0) ? tau - (lam[j] - lam[o]) : tau - lam[j];
    double s = 0.0;
    for (int64_t a = 0; a < k; ++a) s += u[a] * c[a];
    w[j] = s / y;
    nrm += w[j] * w[j];
  }
  nrm = sqrt(nrm);
  for (int64_t j = 0; j < n; ++j) w[j] /= nrm;
  sign_and_store(n, w);
}

int eigref_eigvecs(int64_t n, int64_t k, const double *lam, const double *U,
                   const int8_t *sigma, int64_t nvec, const int64_t *origin, const double *tau,
                   const int64_t *cluster, const int64_t *mult, double *W, int64_t ldw) {
  if (check_common(n, k, lam, U, sigma) != REF_OK || nvec < 0 || !origin || !tau || !W ||
      ldw < n)
    return REF_EINVAL;
  int err = REF_OK;
#pragma omp parallel
  {
    double *buf = (double *)malloc(sizeof(double) * (size_t)(3 * k * k + k));
    if (!buf) {
#pragma omp atomic write
      err = REF_ENOMEM;
    }
#pragma omp for schedule(dynamic, 4)
    for (int64_t t = 0; t < nvec; ++t) {
      if (!buf) continue;
      one_vector(n, k, lam, U, sigma, origin[t], tau[t], cluster ? cluster[t] : 0,
                 mult ? mult[t] : 1, buf, buf + k * k, buf + 3 * k * k, buf + 2 * k * k,
                 W + t * ldw);
    }
    free(buf);
  }
  return err;
}

/* ------------------------------------------------------------------------ */
/* Plain blocked GEMM: C = A B, all column-major (A m-by-kk, B kk-by-nn).    */
/* ------------------------------------------------------------------------ */
int eigref_gemm(int64_t m, int64_t nn, int64_t kk, const double *A, int64_t lda,
                const double *B, int64_t ldb, double *C, int64_t ldc) {
  if (m < 0 || nn < 0 || kk < 0 || lda < m || ldb < kk || ldc < m) return REF_EINVAL;
  const int64_t BJ = 64, BL = 256;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t j0 = 0; j0 < nn; j0 += BJ) {
    int64_t j1 = j0 + BJ < nn ? j0 + BJ : nn;
    for (int64_t j = j0; j < j1; ++j)
      for (int64_t i = 0; i < m; ++i) C[i + j * ldc] = 0.0;
    for (int64_t l0 = 0; l0 < kk; l0 += BL) {
      int64_t l1 = l0 + BL < kk ? l0 + BL : kk;
      for (int64_t j = j0; j < j1; ++j)
        for (int64_t l = l0; l < l1; ++l) {
          double b = B[l + j * ldb];
          if (b == 0.0) continue;
          const double *a = A + l * lda;
          double *c = C + j * ldc;
          for (int64_t i = 0; i < m; ++i) c[i] += a[i] * b;
        }
    }
  }
  return REF_OK;
}

/* ------------------------------------------------------------------------ */
/* The whole update.  lam ascending (ties allowed), Q n-by-n column-major,   */
/* K n-by-k column-major, sigma +-1.  Writes the n updated eigenvalues       */
/* ascending to lam_out and, unless values_only, the updated eigenvectors to */
/* Q_out (n-by-n column-major, ldqo) and the Q-basis eigenvectors to W_out   */
/* (optional, n-by-n column-major, leading dimension n).                     */
/* Exactly-zero rows of U are deflated: their eigenpair is (lam_j, e_j).     */
/* A run of consecutive nonzero-row roots whose values agree to within        */
/* 4 eps (|lam|_max + ||U||_F^2) and that share one origin pole is treated   */
/* as one multiple eigenvalue (see eigref_eigvecs).                           */
/* ------------------------------------------------------------------------ */
int eigref_update(int64_t n, int64_t k, const double *lam, const double *Q, int64_t ldq,
                  const double *K, int64_t ldk, const int8_t *sigma, int32_t values_only,
                  double *lam_out, double *Q_out, int64_t ldqo, double *W_out) {
  if (n < 1 || k < 1 || k > 64 || !lam || !Q || !K || !sigma || !lam_out || ldq < n ||
      ldk < n)
    return REF_EINVAL;
  if (!values_only && (!Q_out || ldqo < n)) return REF_EINVAL;
  double *U = (double *)malloc(sizeof(double) * (size_t)(n * k));
  if (!U) return REF_ENOMEM;
  int err = eigref_qtk(n, k, Q, ldq, K, ldk, U);
  if (err == REF_OK) err = check_common(n, k, lam, U, sigma);
  if (err != REF_OK) {
    free(U);
    return err;
  }
  /* split rows: zero rows (deflated) and the reduced problem */
  int64_t nz = 0, nr = 0;
  int64_t *zrow = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  int64_t *rrow = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  double *lr = (double *)malloc(sizeof(double) * (size_t)n);
  double *Ur = (double *)malloc(sizeof(double) * (size_t)(n * k));
  double *rv = (double *)malloc(sizeof(double) * (size_t)n);
  double *rt = (double *)malloc(sizeof(double) * (size_t)n);
  int64_t *ro = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  int64_t *rc = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  int64_t *rm = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  int64_t *colsrc = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  double *W = NULL;
  if (!values_only) W = (double *)calloc((size_t)(n * n), sizeof(double));
  if (!zrow || !rrow || !lr || !Ur || !rv || !rt || !ro || !rc || !rm || !colsrc ||
      (!values_only && !W)) {
    err = REF_ENOMEM;
    goto done;
  }
  for (int64_t j = 0; j < n; ++j) {
    if (row_is_zero(k, U + j * k)) {
      zrow[nz++] = j;
    } else {
      lr[nr] = lam[j];
      memcpy(Ur + nr * k, U + j * k, sizeof(double) * (size_t)k);
      rrow[nr++] = j;
    }
  }
  if (nr > 0) {
    err = eigref_eigvals(nr, k, lr, Ur, sigma, nr, NULL, rv, ro, rt, NULL);
    if (err != REF_OK) goto done;
  }
  {
    double amax = 0.0, fro = 0.0;
    for (int64_t j = 0; j < n; ++j) amax = fmax(amax, fabs(lam[j]));
    for (int64_t a = 0; a < n * k; ++a) fro += U[a] * U[a];
    double tol = 4.0 * EPS * (amax + fro);
    /* runs of equal roots within one pole interval */
    int64_t s = 0;
    while (s < nr) {
      int64_t e = s + 1;
      while (e < nr && ro[e] == ro[s] && fabs(rv[e] - rv[e - 1]) <= tol) ++e;
      for (int64_t t = s; t < e; ++t) {
        rc[t] = t - s;
        rm[t] = e - s;
      }
      s = e;
    }
  }
  /* merge: zero-row eigenvalues first on ties */
  {
    int64_t a = 0, b = 0, pos = 0;
    while (a < nz || b < nr) {
      if (b >= nr || (a < nz && lam[zrow[a]] <= rv[b])) {
        lam_out[pos] = lam[zrow[a]];
        colsrc[pos++] = -1 - a;
        ++a;
      } else {
        lam_out[pos] = rv[b];
        colsrc[pos++] = b;
        ++b;
      }
    }
  }
  if (!values_only) {
    double *Wr = NULL;
    if (nr > 0) {
      Wr = (double *)malloc(sizeof(double) * (size_t)(nr * nr));
      if (!Wr) {
        err = REF_ENOMEM;
        goto done;
      }
      err = eigref_eigvecs(nr, k, lr, Ur, sigma, nr, ro, rt, rc, rm, Wr, nr);
      if (err != REF_OK) {
        free(Wr);
        goto done;
      }
    }
    for (int64_t p = 0; p < n; ++p) {
      double *col = W + p * n;
      if (colsrc[p] < 0) {
        col[zrow[-1 - colsrc[p]]] = 1.0;
      } else {
        const double *wr = Wr + colsrc[p] * nr;
        for (int64_t t = 0; t < nr; ++t) col[rrow[t]] = wr[t];
      }
    }
    free(Wr);
    err = eigref_gemm(n, n, n, Q, ldq, W, n, Q_out, ldqo);
    if (W_out) memcpy(W_out, W, sizeof(double) * (size_t)(n * n));
  }
done:
  free(U);
  free(zrow);
  free(rrow);
  free(lr);
  free(Ur);
  free(rv);
  free(rt);
  free(ro);
  free(rc);
  free(rm);
  free(colsrc);
  free(W);
  return err;
}
