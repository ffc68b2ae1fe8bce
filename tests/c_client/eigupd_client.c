/* A plain C client of the C ABI (include/eigupd.h): one rank-2 update of a
 * resident decomposition, checked on the host.  It needs only the HIP runtime's
 * C API for device memory, no Python and no torch.
 *
 * A = diag(lambda) (Q = I), A' = A + K Sigma K^T with K = [(e_j + a)/sqrt2,
 * (e_j - a)/sqrt2], Sigma = diag(1, -1) -- the rank-2 update e_j a^T + a e_j^T
 * of Sec. 2.2.  Checks: eigenvalues ascending; trace(A') = sum(lambda') (the
 * trace identity); max|Q'^T Q' - I| and max|A' Q' - Q' Lambda'| / ||A'|| small.
 * Exit status 0 when every check passes. */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "eigupd.h"

#define N 96

static uint64_t rng_state = 12345u;
static double uniform(void) { /* splitmix64 -> [0, 1) */
  uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

#define CHECK(cond, ...)          \
  do {                            \
    if (!(cond)) {                \
      fprintf(stderr, __VA_ARGS__); \
      return 1;                   \
    }                             \
  } while (0)

int main(void) {
  const int n = N, k = 2, j = 17;
  static double lam[N], Q[N * N], K[N * 2], lam_out[N], Q_out[N * N], A[N * N];
  double a[N];
  for (int i = 0; i < n; ++i) lam[i] = -1.0 + 2.0 * (i + 0.25 + 0.5 * uniform()) / n;
  for (int i = 0; i < n * n; ++i) Q[i] = 0.0;
  for (int i = 0; i < n; ++i) Q[i * n + i] = 1.0;
  for (int i = 0; i < n; ++i) a[i] = (uniform() - 0.5) / sqrt((double)n);
  for (int i = 0; i < n; ++i) {
    const double e = (i == j) ? 1.0 : 0.0;
    K[i] = (e + a[i]) / sqrt(2.0);     /* column 0, sigma = +1 */
    K[n + i] = (e - a[i]) / sqrt(2.0); /* column 1, sigma = -1 */
  }
  const int8_t sigma[2] = {1, -1};

  double *dlam, *dQ, *dK;
  CHECK(hipMalloc((void**)&dlam, sizeof lam) == hipSuccess, "hipMalloc failed\n");
  CHECK(hipMalloc((void**)&dQ, sizeof Q) == hipSuccess, "hipMalloc failed\n");
  CHECK(hipMalloc((void**)&dK, sizeof K) == hipSuccess, "hipMalloc failed\n");
  CHECK(hipMemcpy(dlam, lam, sizeof lam, hipMemcpyHostToDevice) == hipSuccess, "copy\n");
  CHECK(hipMemcpy(dQ, Q, sizeof Q, hipMemcpyHostToDevice) == hipSuccess, "copy\n");
  CHECK(hipMemcpy(dK, K, sizeof K, hipMemcpyHostToDevice) == hipSuccess, "copy\n");

  eig_state_t s = NULL;
  int rc = eig_state_create(&s, n, 0);
  CHECK(rc == EIG_OK, "eig_state_create: %s\n", eig_status_str(rc));
  rc = eig_state_upload(s, dlam, dQ, n, 1, NULL);
  CHECK(rc == EIG_OK, "eig_state_upload: %s\n", eig_status_str(rc));
  rc = eig_update_rankk(s, k, dK, n, sigma, EIG_GEMM_FP64, NULL);
  CHECK(rc == EIG_OK, "eig_update_rankk: %s\n", eig_status_str(rc));
  eig_info info;
  rc = eig_query(s, lam_out, Q_out, n, 0, &info, NULL);
  CHECK(rc == EIG_OK, "eig_query: %s\n", eig_status_str(rc));
  eig_state_destroy(s);
  hipFree(dlam);
  hipFree(dQ);
  hipFree(dK);

  /* A' = diag(lambda) + K Sigma K^T (column-major) */
  double anorm = 0.0, tr = 0.0, tr_out = 0.0;
  for (int c = 0; c < n; ++c)
    for (int r = 0; r < n; ++r) {
      double v = (r == c) ? lam[r] : 0.0;
      v += K[r] * K[c] - K[n + r] * K[n + c];
      A[c * n + r] = v;
      anorm = fmax(anorm, fabs(v));
    }
  for (int i = 0; i < n; ++i) {
    tr += A[i * n + i];
    tr_out += lam_out[i];
  }
  for (int i = 1; i < n; ++i) CHECK(lam_out[i - 1] <= lam_out[i], "eigenvalues not ascending\n");
  CHECK(fabs(tr - tr_out) <= 1e-12 * n * anorm, "trace %.17g vs %.17g\n", tr, tr_out);
  double orth = 0.0, res = 0.0;
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q) {
      double d = 0.0;
      for (int r = 0; r < n; ++r) d += Q_out[p * n + r] * Q_out[q * n + r];
      orth = fmax(orth, fabs(d - (p == q ? 1.0 : 0.0)));
    }
  for (int c = 0; c < n; ++c)
    for (int r = 0; r < n; ++r) {
      double d = 0.0;
      for (int t = 0; t < n; ++t) d += A[t * n + r] * Q_out[c * n + t];
      res = fmax(res, fabs(d - lam_out[c] * Q_out[c * n + r]));
    }
  CHECK(orth <= 1e-12, "orthogonality %.3e\n", orth);
  CHECK(res <= 1e-12 * anorm, "residual %.3e\n", res);
  printf("c client ok: n=%d k=%d orth %.2e residual %.2e iters %.1f\n", n, k, orth, res / anorm,
         info.iters_mean);
  return 0;
}
