/*
 * eigupd.h -- C ABI of the MI355X rank-k symmetric eigen-update library
 * (libeigupd.so, HIP kernels for gfx950).
 *
 * Method: Oh & Hu, "Multiple-rank Modification of Symmetric Eigenvalue
 * Problem" (arXiv:1706.00773).  Given a resident decomposition
 * A = Q diag(lambda) Q^T (Sec. 2.1) and a perturbation K Sigma K^T, K n-by-k,
 * Sigma = diag(sigma_c) with sigma_c = +-1 (the paper's K K^T of Sec. 2.1 and
 * the one-column-one-row form e_j a^T + a e_j^T of Sec. 2.2, Steps 1-2, which
 * is k = 2, Sigma = diag(1, -1)), one update computes the eigen-decomposition
 * of A' = A + K Sigma K^T:
 *   U = Q^T K                                 (Sec. 2.1, below eq. (1))
 *   all n roots of det(I_k - Sigma U^T (xI - diag(lambda))^{-1} U) = 0
 *     (eq. (1)), located per pole interval by an inertia count that plays
 *     the role of the modified Sturm chain (Sec. 2.2) and refined by
 *     safeguarded Newton/bisection (the zero finder of Sec. 2.3)
 *   eigenvectors w = (lambda' I - diag(lambda))^{-1} U c, normalised
 *     (Sec. 2.4, eq. (10)), back-transformed Q' = Q W.
 * Everything runs in FP64 on the device unless a reduced-precision mode is
 * asked for (see the mode bits).
 *
 * Conventions common to all entry points
 *   - Matrices are column-major.  lambda is ascending.
 *   - A state is bound to one device for its lifetime and is not
 *     thread-safe; distinct states may be used concurrently.
 *   - `hip_stream` is a hipStream_t (NULL = the default stream).  Work is
 *     enqueued on it in stream order.  Device pointers passed in are
 *     borrowed until the stream reaches the work that reads them; host
 *     pointers are copied before the call returns.
 *   - Every entry point returns an eig_status code (EIG_OK = 0).  Argument
 *     errors are reported synchronously and leave the state unchanged.
 *     Errors detected on the device (non-finite input, non-convergence) are
 *     deferred: they are sticky, every later update on the state becomes a
 *     no-op on the device, and the next eig_query reports the first one,
 *     clears it and leaves the state at its last committed decomposition.
 */
#ifndef EIGUPD_H
#define EIGUPD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct eig_state_s *eig_state_t;

/* Per-update diagnostics returned by eig_query (values of the last update). */
typedef struct {
  int64_t n;                 /* order of the matrix */
  int64_t k;                 /* rank of the last update */
  int64_t p, q;              /* number of sigma_c = +1 and = -1 */
  int64_t n_deflated_rows;   /* eigenpairs deflated (tiny rows of U, equal-pole groups) */
  int64_t n_deflated_groups; /* near-equal pole groups of two or more rows */
  int64_t n_segments;        /* distinct poles of the reduced secular problem */
  int32_t iters_min;         /* count/Newton evaluations per root */
  int32_t iters_max;
  double iters_mean;
  double defl_backward_err;  /* bound on ||perturbation|| introduced by deflation */
  double anorm_bound;        /* max|lambda| + ||U||_F^2 >= ||A'||_2 */
  int64_t generation;        /* updates committed since the last upload */
  double ms[8];              /* phase times of the last update in milliseconds when it ran
                                with EIG_PHASE_TIMING (else 0): [0] Q^T K, [1] deflation,
                                [2] pole counts and location, [3] root refinement and null
                                vectors, [4] eigenvalue merge and W, [5] Q W, [6] commit,
                                [7] whole update */
  int32_t located_by_residues; /* 1 if the roots were located by residue signs */
  int32_t reserved;
} eig_info;

/* Status codes. */
enum {
  EIG_OK = 0,
  EIG_EINVAL = -1,       /* invalid argument */
  EIG_ENOMEM = -2,       /* device allocation failed */
  EIG_EDEVICE = -3,      /* HIP runtime error or no such device */
  EIG_ENOCONV = -4,      /* a root did not converge within the evaluation cap */
  EIG_ENOTSORTED = -5,   /* uploaded lambda not ascending */
  EIG_EUNSUPPORTED = -6, /* k beyond EIG_KMAX or a mode not built */
  EIG_EDEPENDENCY = -7,  /* serving: an earlier update of the matrix failed */
  EIG_ESTATE = -8,       /* state not uploaded */
  EIG_ENONFINITE = -9,   /* NaN or Inf in an input or in U */
  EIG_ECHECK = -10       /* a check of EIG_DEBUG_CHECKS failed */
};

/* Mode bits of eig_update_rankk.  Bits 0-1 select the arithmetic of the two
 * dense products U = Q^T K and Q' = Q W; the secular roots, the pole
 * differences and the deflation tests are FP64 in every mode.
 *   EIG_GEMM_FP64         both products in FP64 (FP64 matrix cores for Q W).
 *   EIG_GEMM_FP32_CORR    operands split x = hi + lo into two FP32 numbers;
 *                         Q W = hi*hi + (hi*lo + lo*hi) on FP32 matrix cores
 *                         with FP32 accumulation, the partial sums of every
 *                         16-deep k-slice added up in FP64.
 *   EIG_GEMM_BF16X3_CORR  operands split into three bfloat16 numbers; the six
 *                         products b_i*b_j with i + j <= 2 on BF16 matrix
 *                         cores with FP32 accumulation, every 32-deep k-slice
 *                         added up in FP64.
 * In both reduced modes U is formed the same way (on the vector units) and
 * then corrected once in FP64: U = U0 + lo(Q^T (K - Q U0)) with K - Q U0
 * formed in FP64, which brings U back to FP64 accuracy.  The eigenvectors
 * carry the rounding of the reduced Q W (about 1e-7 relative); the
 * eigenvalues do not.  Q and W are split once per update into slice planes:
 * the first update of a state in a reduced mode (without EIG_VALUES_ONLY)
 * allocates them, 12 n^2 bytes for BF16X3 and 16 n^2 bytes for FP32, and the
 * state keeps them until eig_state_destroy (a later update that needs more
 * synchronises the device and reallocates). */
enum {
  EIG_GEMM_FP64 = 0,
  EIG_GEMM_FP32_CORR = 1,
  EIG_GEMM_BF16X3_CORR = 2,
  EIG_GEMM_MASK = 3,
  EIG_VALUES_ONLY = 1 << 4, /* eigenvalues only: nothing is committed, eig_query
                               returns these values until the next update */
  EIG_DEBUG_CHECKS = 1 << 5, /* after the update and before its commit, check on
                                the device: the new eigenvalues ascend, each lies
                                in its Courant-Weyl window [lambda_{i-q},
                                lambda_{i+p}] (Sec. 2.2) and their sum changes by
                                sum_c sigma_c ||U_c||^2 (the trace of K Sigma
                                K^T); unless values-only, 8 sampled columns of W
                                solve the eigenproblem of diag(lambda) + U Sigma
                                U^T (Sec. 2.4, eq. (10)) to 1e-9 ||A'|| and are
                                orthonormal to 1e-9 (not with EIG_QW_FARFIELD,
                                whose W is partial), and the same columns of Q'
                                are orthonormal to 1e-9 (FP64) or 8e-6 sqrt(n)
                                (reduced modes).  A failed check is the deferred
                                error EIG_ECHECK: nothing is committed.  One
                                small extra kernel; a non-orthogonal uploaded Q
                                is the usual cause */
  EIG_HOST_INPUT = 1 << 6,  /* K is a host pointer (copied before return) */
  EIG_PHASE_TIMING = 1 << 7, /* record HIP events between the phases on hip_stream;
                                eig_query reports the times in eig_info.ms */
  EIG_LOCATE_RESIDUES = 1 << 8, /* k = 2: locate the roots by the signs of the
                                  residues alpha_i (Sec. 2.2, eq. (2), Alg. 1a-1c)
                                  instead of the inertia pole counts; taken only
                                  when every pole is simple and every residue is
                                  larger than its rounding bound, else the pole
                                  counts run (eig_info.located_by_residues tells
                                  which); ignored for k != 2 */
  EIG_QW_FARFIELD = 1 << 9  /* FP64, n >= 2048: form Q' = Q W with the far blocks
                               of W (Sec. 2.4, eq. (10)) replaced by Chebyshev
                               expansions of 1/(x - y) (column blocks of 256;
                               row blocks of 128 up to k = 2, of 256 above): a
                               band of exact block products plus three small
                               products, about 9.8x fewer flops at n = 8192,
                               k = 2.  A row block and a column block count as
                               far when their distance is at least etac times
                               the column block's width and etar times the row
                               block's; there the interpolant of 1/(x - y)
                               errs by at most about 3e-13 relative up to
                               k = 2 (etac 0.45 with 24 nodes, etar 0.85 with
                               20) and about 6e-14 above (0.78 of either width,
                               20 nodes), and by about 2e-15 for blocks one
                               width apart.  The far entries of W are small next to
                               the near ones, so Q' agrees with the dense
                               product to about 1e-15 in practice.
                               Falls back to the dense
                               product on the device when the update merged
                               equal poles; ignored for n < 2048, for
                               n >= 2049 * 256 and with the
                               reduced-precision modes; batches take it too
                               (eig_update_batch).  Only the blocks of W
                               it reads are formed (the debug copy of W is then
                               partial).  Allocates its buffers (about
                               2 k n^2 20 / 256 doubles from k = 3, about
                               k n^2 (20 / 128 + 24 / 256) up to k = 2) on
                               first use. */
};

/* Ranks: the kernels are specialised for 1 <= k <= EIG_KMAX.  eig_update_rankk
 * also takes EIG_KMAX < k <= EIG_KMAX_GENERIC: the update is then applied as
 * ceil(k / EIG_KMAX) successive updates of nearly equal rank (A + K Sigma K^T =
 * (A + K_1 Sigma_1 K_1^T) + K_2 Sigma_2 K_2^T + ...; the paper's Sec. 3 compares
 * exactly this split, two rank-1 updates, with one rank-2 update).  The other
 * entry points take k <= EIG_KMAX. */
enum { EIG_KMAX = 8, EIG_KMAX_GENERIC = 32 };

/* Create a state for matrices of order n on HIP device `device`, and allocate
 * all its device memory: two copies of (lambda, Q) used alternately, the
 * n-by-n eigenvector matrix W and O(n * EIG_KMAX) of workspace -- about
 * 24 n^2 bytes.  Only the first reduced-precision update allocates more
 * (the slice planes described at the mode bits); no other call does.
 * Errors: EIG_EINVAL (out NULL, n < 1), EIG_EDEVICE, EIG_ENOMEM.
 * On success *out owns the memory until eig_state_destroy. */
int eig_state_create(eig_state_t *out, int64_t n, int32_t device);

/* Knobs of a state (eig_state_set).
 *   EIG_KNOB_MAX_EVALS  evaluations (count and Newton steps together) allowed
 *                       per root before the zero finder of Sec. 2.3 gives up
 *                       and the update fails with the deferred EIG_ENOCONV;
 *                       1 <= value <= 1000000, default 160.  Applies to the
 *                       updates enqueued after the call.
 * Errors: EIG_EINVAL (unknown knob, value out of range). */
enum { EIG_KNOB_MAX_EVALS = 6 };
int eig_state_set(eig_state_t s, int32_t knob, int64_t value);

/* Load a decomposition: lambda (n values, ascending, ties allowed) and Q
 * (n-by-n column-major, leading dimension ldq >= n, columns orthonormal).
 * ptrs_on_device != 0: both are device pointers on the state's device.
 * The call synchronises `hip_stream`.  Resets the generation to 0 and clears
 * any deferred error.  Errors: EIG_EINVAL, EIG_ENOTSORTED (lambda descends
 * somewhere or is not finite), EIG_EDEVICE. */
int eig_state_upload(eig_state_t s, const double *lambda, const double *Q, int64_t ldq,
                     int32_t ptrs_on_device, void *hip_stream);

/* Apply A' = A + K Sigma K^T to the resident decomposition (Sec. 2.1-2.4).
 *   k      rank, 1 <= k <= min(n, EIG_KMAX_GENERIC).  For k > EIG_KMAX the
 *          update runs as ceil(k / EIG_KMAX) chained parts; every part reads
 *          the previous part's (lambda, Q), the committed pair is only read,
 *          and the whole update commits at once (a device error in any part
 *          leaves the state unchanged).  The first such update allocates one
 *          more n-by-n buffer (8 n^2 bytes), kept until eig_state_destroy.
 *          eig_info then describes the last part (its deflation, counts and
 *          evaluations; p and q are the whole update's), eig_info.ms[0] also
 *          holds the earlier parts, and eig_debug_fetch returns the last
 *          part's intermediates (EIG_DBG_U: EIG_EINVAL).
 *   K      n-by-k column-major, leading dimension ldk >= n; a device pointer
 *          unless mode has EIG_HOST_INPUT
 *   sigma  host array of k entries, each +1 or -1
 *   mode   one of EIG_GEMM_FP64, EIG_GEMM_FP32_CORR, EIG_GEMM_BF16X3_CORR,
 *          optionally | EIG_VALUES_ONLY | EIG_HOST_INPUT | EIG_PHASE_TIMING
 *          | EIG_LOCATE_RESIDUES | EIG_QW_FARFIELD | EIG_DEBUG_CHECKS
 * Asynchronous: enqueues the kernels on `hip_stream` and returns.  On the
 * device the update writes the new pair into the state's other buffer and
 * commits it only if no error was raised; the state then holds A'.
 * Errors (synchronous): EIG_EINVAL, EIG_EUNSUPPORTED (k > EIG_KMAX_GENERIC,
 * an unknown mode bit, or precision selector 3), EIG_ENOMEM (slice planes of
 * a reduced mode, the far-field buffers or the chained parts' buffer could not
 * be allocated),
 * EIG_ESTATE (no upload yet), EIG_EDEVICE (launch failure).  Deferred:
 * EIG_ENONFINITE, EIG_ENOCONV, EIG_ECHECK (see the file header). */
int eig_update_rankk(eig_state_t s, int64_t k, const double *K, int64_t ldk,
                     const int8_t *sigma, uint32_t mode, void *hip_stream);

/* A subset of the spectrum: the eigenpairs of A' = A + K Sigma K^T whose
 * eigenvalues lie in [a, b), without changing the state (Sec. 2.1: when only
 * the eigenvalues in an interval are of interest, the first sub-problem -- the
 * count -- is enough; Sec. 3: a subset of eigenvectors, e.g. a null space, is
 * much cheaper than a full decomposition).  The counts at a and b select the
 * roots of the secular equation to refine; only those m roots are solved and
 * V = Q W is an n x n by n x m product (2 n^2 m flops instead of 2 n^3).
 *   k, K, ldk, sigma   as for eig_update_rankk (K a device pointer unless
 *                      mode has EIG_HOST_INPUT)
 *   a <= b             the interval (infinite ends allowed); eigenvalues within
 *                      rounding of a or b may fall on either side
 *   mode               optional EIG_VALUES_ONLY | EIG_HOST_INPUT |
 *                      EIG_LOCATE_RESIDUES
 *   lambda_out         device pointer, m_max doubles: the m eigenvalues, ascending
 *   V_out              device pointer, n-by-m_max column-major, leading dimension
 *                      ldv >= n: their unit eigenvectors (not used with
 *                      EIG_VALUES_ONLY)
 *   *m_out             m, the number of eigenvalues in [a, b)
 * Synchronous: returns after the outputs are written.  If m > m_max nothing is
 * written, *m_out is m and the call returns EIG_EINVAL (call again with room).
 * Errors: as eig_update_rankk; a device error (non-finite input,
 * non-convergence) is returned directly and cleared. */
int eig_update_interval(eig_state_t s, int64_t k, const double *K, int64_t ldk,
                        const int8_t *sigma, double a, double b, uint32_t mode,
                        double *lambda_out, double *V_out, int64_t ldv, int64_t m_max,
                        int64_t *m_out, void *hip_stream);

/* The first-order perturbation estimate of the eigenpairs of A + K Sigma K^T
 * (Sec. 3, eq. (11), the comparator of the paper's accuracy experiment):
 *   lambda_j ~ lambda_j + u_j^T Sigma u_j,
 *   v_j ~ v_j + sum_{i != j} (u_i^T Sigma u_j) / (lambda_j - lambda_i) v_i
 * (eq. (11) as read: v_i inside the sum, this sign of the denominator, Sigma
 * included; pairs with equal eigenvalues get no first-order term).  Writes
 * lambda_out (n, device) and V_out (n-by-n column-major, device, leading
 * dimension ldv) in the order of the resident eigenvalues; nothing is
 * committed.  Only valid for a perturbation small against the eigenvalue gaps.
 * mode: 0 or EIG_HOST_INPUT.  Asynchronous; errors as eig_update_rankk
 * (deferred ones reported by eig_query). */
int eig_perturb_first_order(eig_state_t s, int64_t k, const double *K, int64_t ldk,
                            const int8_t *sigma, uint32_t mode, double *lambda_out,
                            double *V_out, int64_t ldv, void *hip_stream);

/* The secular Sturm chain of the update A' = A + K Sigma K^T (Sec. 2.2,
 * eqs. (4)-(9)) as an eigenvalue counter, without changing the state.
 * The reduced secular function f_0(x) = 1 - sum_j alpha_j / (x - d_j) (its
 * residues alpha_j are eq. (2)) gives the polynomial p_0 = f_0 prod (x - d_j);
 * each member p_m of its Sturm sequence is kept in secular form (c_m and
 * N - m residues; the division step with the B_m of the long division taken
 * with its sign corrected).  The build stops at the first c_m that is not
 * positive, as the section prescribes: the chain is then partial and only a
 * lower bound on the number of zeros.  Known eigenvalues xi (e.g. found
 * earlier) are divided out first by eq. (9), each removing one of the lowest
 * poles, which leaves a shorter chain.
 *   k, K, ldk, sigma   as for eig_update_rankk (K a device pointer)
 *   xi, n_xi           device pointer: n_xi known eigenvalues of the reduced
 *                      problem (none of them a pole), strictly ascending; may
 *                      be NULL when n_xi == 0
 *   x, n_x             device pointer: the points to count at
 *   counts             device pointer, n_x entries: eigenvalues of A' below
 *                      x[i] (the chain's count, plus the known and the deflated
 *                      eigenvalues below x[i]); -1 where x[i] is a pole of the
 *                      chain.  Exact only when info->complete is 1.
 *   c_out, c_max       device pointer (may be NULL when c_max == 0): the first
 *                      min(c_max, info->levels) leading constants c_m
 *   info               host pointer: the chain's size and state
 * The reduced problem must have simple poles (no two kept rows at one
 * eigenvalue after deflation); otherwise EIG_EUNSUPPORTED.  The members are
 * held in the state's eigenvector work buffer (about N^2 / 2 doubles).
 * Synchronous.  Errors: EIG_EINVAL (arguments, n_xi > N, xi not ascending or
 * on a pole), EIG_EUNSUPPORTED, EIG_ESTATE, EIG_ENOMEM, EIG_EDEVICE, and a
 * device error (a non-finite input) returned directly and cleared. */
typedef struct eig_chain_info {
  int64_t n_poles;     /* N: poles of the chain (the reduced problem's, less n_xi) */
  int64_t levels;      /* members p_0 .. p_{levels-1} built */
  int64_t lower_bound; /* zeros the leading positive c's guarantee: their number - 1 */
  int64_t n_deflated;  /* eigenvalues deflated before the chain (tiny rows, groups) */
  int32_t complete;    /* 1: all N + 1 members, every c_m > 0: the counts are exact */
  int32_t reserved;
} eig_chain_info;

int eig_sturm_chain(eig_state_t s, int64_t k, const double *K, int64_t ldk,
                    const int8_t *sigma, const double *xi, int64_t n_xi, const double *x,
                    int64_t n_x, int64_t *counts, double *c_out, int64_t c_max,
                    eig_chain_info *info, void *hip_stream);

/* Synchronise `hip_stream`, report any deferred error, and copy out the
 * committed decomposition: lambda_out (n values, ascending; may be NULL) and
 * Q_out (n-by-n column-major, leading dimension ldq >= n; may be NULL).
 * Columns of Q_out are unit eigenvectors; in the Q basis each one's
 * component at its root's nearest pole is positive.  ptrs_on_device != 0:
 * the outputs are device pointers.  info may be NULL.
 * If the last update used EIG_VALUES_ONLY, lambda_out receives its values.
 * Returns the deferred error if one was raised (outputs then hold the last
 * committed decomposition), else EIG_OK. */
int eig_query(eig_state_t s, double *lambda_out, double *Q_out, int64_t ldq,
              int32_t ptrs_on_device, eig_info *info, void *hip_stream);

/* Release all device memory of the state (after synchronising the device). */
int eig_state_destroy(eig_state_t s);

/* Static, human-readable text for a status code. */
const char *eig_status_str(int status);

/* ------------------------------------------------------------------ batches
 * Many updates at once: one update of each of several states (their n and k
 * may all differ), applied with every phase launched once per distinct k (or
 * once in all, for Q' = Q W) over descriptor arrays, the root solve possibly
 * as a persistent kernel drawing (state, block of 32 roots) items from a
 * queue, and the whole sequence replayed as a HIP graph for every batch of an
 * already-seen shape.  Each state's result is bitwise the same as with
 * eig_update_rankk.  This is a throughput form of Sec. 2.1-2.4 for serving
 * many decompositions; the paper treats one matrix at a time. */
typedef struct eig_batch_s *eig_batch_t;

typedef struct {
  eig_state_t state;      /* each state at most once per batch */
  int64_t k;              /* 1 <= k <= min(n, EIG_KMAX) */
  const double *K;        /* device pointer, n-by-k column-major */
  int64_t ldk;            /* >= n */
  int8_t sigma[EIG_KMAX]; /* first k entries used, each +1 or -1 */
} eig_batch_item;

/* Create a batch context for up to max_items updates per call on `device`.
 * It owns a small device area for the per-call descriptors, two pinned host
 * staging buffers, a private capture stream and the graph cache.
 * Errors: EIG_EINVAL, EIG_EDEVICE, EIG_ENOMEM. */
int eig_batch_create(eig_batch_t *out, int32_t max_items, int32_t device);

/* Enqueue one update per item on hip_stream (asynchronous, like
 * eig_update_rankk; K borrowed until the stream reaches the batch).  mode:
 * EIG_GEMM_FP64, optionally | EIG_VALUES_ONLY (then nothing is committed and
 * eig_query returns the values, as for a single update) or | EIG_QW_FARFIELD
 * (items with n >= 2048 form Q' by the far-field product, with launches of
 * their own, bitwise as a single update in that mode; the first such update
 * of a state allocates its far-field buffers, sized for rank EIG_KMAX; a
 * batch with such items is launched directly, never replayed as a graph).
 * A shape -- the
 * ordered (k, n) list and the mode -- is tuned on its first two calls (those
 * two synchronise the stream) and captured into a HIP graph on its next call;
 * later calls with that shape replay the graph.  Calls on one batch context
 * must be serialised on one stream.  Device errors are per state (sticky in
 * that state, reported by its eig_query); the other states commit.
 * Errors (synchronous, nothing enqueued): EIG_EINVAL (bad item, a state twice,
 * count out of range, a state on another device), EIG_ESTATE (a state not
 * uploaded), EIG_EUNSUPPORTED (k > EIG_KMAX or other mode bits), EIG_ENOMEM (the
 * far-field buffers), EIG_EDEVICE. */
int eig_update_batch(eig_batch_t b, const eig_batch_item *items, int32_t count, uint32_t mode,
                     void *hip_stream);

/* Knobs (eig_batch_set) and read-outs (eig_batch_get) of a batch context.
 *   EIG_KNOB_ROOTSOLVE   EIG_AUTO (tuned), EIG_ROOTSOLVE_GROUPED (one block per
 *                        item), EIG_ROOTSOLVE_PERSISTENT (queue); get: the form
 *                        the last call used
 *   EIG_KNOB_GEMM_TILE   EIG_AUTO, 64 or 128; get: the tile the last call used
 *   EIG_KNOB_GRAPHS      1 (default) capture and replay graphs, 0 never; get:
 *                        1 if the last call replayed a graph
 *   EIG_STAT_GRAPH_LAUNCHES, EIG_STAT_GRAPHS_CACHED (get only)
 * Errors: EIG_EINVAL. */
enum {
  EIG_KNOB_ROOTSOLVE = 1,
  EIG_KNOB_GEMM_TILE = 2,
  EIG_KNOB_GRAPHS = 3,
  EIG_STAT_GRAPH_LAUNCHES = 4,
  EIG_STAT_GRAPHS_CACHED = 5
};
enum { EIG_AUTO = 0, EIG_ROOTSOLVE_GROUPED = 1, EIG_ROOTSOLVE_PERSISTENT = 2 };
int eig_batch_set(eig_batch_t b, int32_t knob, int32_t value);
int eig_batch_get(eig_batch_t b, int32_t knob, int64_t *value);

/* Release the context (after synchronising the device). */
int eig_batch_destroy(eig_batch_t b);

/* ------------------------------------------------------------------ serving
 * A request loop over many resident decompositions.  Requests (matrix, k, K,
 * sigma) are submitted from the host at any time; a scheduler thread admits
 * them by device-memory footprint and runs them as batched updates
 * (eig_update_batch) on several streams, starting a new batch on any stream
 * whose previous batch has finished, so batches overlap on the device
 * (continuous batching).  Updates of one matrix run in arrival order, one at a
 * time, each on the decomposition its predecessor committed; a request's
 * result is therefore the same as applying the same updates to that matrix
 * alone.  As on a single state (where a failed update turns the later ones
 * into no-ops until eig_query), a request that fails on the device leaves its
 * matrix unchanged, and every later request of that matrix completes with
 * EIG_EDEPENDENCY without being applied until eig_server_read of that matrix:
 * an update is never applied to a decomposition other than the one its
 * predecessors were meant to produce.
 *
 * Products: batches run with EIG_QW_FARFIELD, so matrices with n >= 2048 form
 * Q' by the far-field product; its buffers (about 2 EIG_KMAX n^2 20 / 256
 * doubles per such matrix, the most over every rank) are allocated outside the
 * arena on the matrix's first update and kept.
 *
 * Memory: one device arena of arena_bytes holds every n x n buffer.  A
 * resident matrix keeps its current Q there (8 n^2 bytes; lambda and O(n k)
 * workspace live outside the arena); an admitted update borrows W and Q'
 * (16 n^2 bytes) until it has finished, then the old Q (or, if the update
 * failed, Q') and W are returned.  A request is admitted when both fit; the
 * oldest waiting request is never overtaken while it waits for memory.  When
 * requests wait with nothing running, the resident Q buffers are packed to
 * one end of the arena first (their contents are moved on the device). */
typedef struct eig_server_s *eig_server_t;

typedef struct {
  int64_t request_id; /* the caller's tag */
  int32_t matrix;
  int32_t status;     /* EIG_OK, or the error of this update (EIG_ENONFINITE,
                         EIG_ENOCONV, EIG_ENOMEM if it could never fit,
                         EIG_EDEPENDENCY if an earlier update of the matrix
                         failed and the matrix was not read since, ...) */
  double t_submit;    /* seconds since eig_server_create */
  double t_admit;     /* its batch was enqueued */
  double t_done;      /* the scheduler saw its batch finish */
  int32_t batch_size; /* updates in that batch */
  int32_t reserved;
} eig_completion;

typedef struct {
  int64_t matrices, submitted, completed, failed, queued, in_flight, batches;
  double mean_batch;                 /* updates per batch */
  int64_t arena_bytes, resident_bytes, arena_used, arena_peak;
  int64_t compactions;               /* times the resident buffers were packed */
} eig_server_info;

/* Create a server on `device`: an arena of arena_bytes, batches of at most
 * max_batch updates, `streams` streams (1-8), and staging for at most
 * max_k_doubles doubles of K per batch (a request needs n*k).
 * Errors: EIG_EINVAL, EIG_EDEVICE, EIG_ENOMEM. */
int eig_server_create(eig_server_t *out, int32_t device, int64_t arena_bytes, int32_t max_batch,
                      int32_t streams, int64_t max_k_doubles);

/* Register a decomposition (lambda ascending, Q n-by-n column-major, leading
 * dimension ldq; device pointers if ptrs_on_device).  Copied; synchronous.
 * *matrix receives its id (0, 1, ...).  Errors: EIG_EINVAL, EIG_ENOTSORTED,
 * EIG_ENOMEM (its Q plus one update of the largest matrix would not fit). */
int eig_server_add(eig_server_t s, int64_t n, const double *lambda, const double *Q, int64_t ldq,
                   int32_t ptrs_on_device, int32_t *matrix);

/* Queue A' = A + K diag(sigma) K^T for `matrix` (K on the host, n-by-k,
 * leading dimension ldk; copied before return).  Errors: EIG_EINVAL,
 * EIG_EUNSUPPORTED (k > EIG_KMAX). */
int eig_server_submit(eig_server_t s, int32_t matrix, int64_t k, const double *K, int64_t ldk,
                      const int8_t *sigma, int64_t request_id);

/* Take up to max completions (waiting up to timeout_ms for the first). */
int eig_server_poll(eig_server_t s, eig_completion *out, int32_t max, int32_t timeout_ms,
                    int32_t *count);

/* Wait until every submitted request has completed. */
int eig_server_drain(eig_server_t s);

/* Copy out a matrix's current decomposition after its queued updates have
 * finished (waits for them).  Clears the matrix's failed mark: requests
 * submitted afterwards are applied again. */
int eig_server_read(eig_server_t s, int32_t matrix, double *lambda_out, double *Q_out,
                    int64_t ldq, int32_t ptrs_on_device);

int eig_server_stats(eig_server_t s, eig_server_info *info);

/* Finish every queued request, then release everything. */
int eig_server_destroy(eig_server_t s);

/* ---------------------------------------------------------- no allocation
 * For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the
 * eigenvalues of A' = A + K Sigma K^T from a decomposition the caller holds,
 * computed by the kernels of eig_update_rankk with EIG_VALUES_ONLY, with no
 * state and no allocation.  The workspace (U, deflation, reduced problem,
 * roots: about 600 bytes per row) lives in one static device array of 10 MiB
 * that each device keeps until the process ends.  Every call on a device
 * shares that device's array and leaves its contents behind: calls that
 * overlap on one device (different streams, or host threads) race and must
 * be serialised by the caller.
 *   n, k          order (1 <= n <= EIG_NOALLOC_NMAX) and rank (1 <= k <=
 *                 min(n, EIG_KMAX))
 *   lambda        device pointer, n values, ascending (ties allowed)
 *   Q             device pointer, n-by-n column-major, leading dimension
 *                 ldq >= n, orthonormal columns
 *   K             device pointer, n-by-k column-major, leading dimension ldk >= n
 *   sigma         host array of k entries, each +1 or -1
 *   mode          0 or EIG_LOCATE_RESIDUES
 *   lambda_out    device pointer, n doubles: the eigenvalues of A', ascending
 *   status_out    device pointer to one int32: EIG_OK, or EIG_ENONFINITE /
 *                 EIG_ENOCONV when the device found a non-finite input or a
 *                 root that did not converge (lambda_out is then unspecified)
 *   device        the HIP device of all pointers
 * Asynchronous: enqueues the kernels on hip_stream (NULL = default stream)
 * and returns; the inputs are read and the outputs written in stream order.
 * Calls no hipMalloc, hipFree or other allocating routine.
 * Errors (synchronous, nothing enqueued): EIG_EINVAL (NULL pointer, n < 1,
 * k < 1, k > n, ld < n, sigma not +-1), EIG_EUNSUPPORTED (n > EIG_NOALLOC_NMAX,
 * k > EIG_KMAX, another mode bit), EIG_EDEVICE (no such device, launch
 * failure). */
enum { EIG_NOALLOC_NMAX = 16384 };
int eig_eigvals_rankk_noalloc(int64_t n, int64_t k, const double *lambda, const double *Q,
                              int64_t ldq, const double *K, int64_t ldk, const int8_t *sigma,
                              uint32_t mode, double *lambda_out, int32_t *status_out,
                              int32_t device, void *hip_stream);

/* Diagnostics: copy an intermediate of the last update to host memory `dst`
 * (`bytes` available) after synchronising `hip_stream`.  `what`:
 *   EIG_DBG_U            U = Q^T K, n-by-k row-major doubles
 *   EIG_DBG_POLE_COUNT   nu at each distinct pole of the reduced problem,
 *                        n_segments int32 (eigenvalues strictly below it)
 *   EIG_DBG_SEG_START    first reduced row of each segment, n_segments+1 int32
 *   EIG_DBG_REDUCED_D    poles of the reduced problem, n-n_deflated doubles
 *   EIG_DBG_REDUCED_ROW  original row of each reduced row, int32
 *   EIG_DBG_ROOT_ORIGIN  segment index of each root's origin pole, int32
 *   EIG_DBG_ROOT_TAU     each root's offset from its origin pole, doubles
 *   EIG_DBG_ROOT_ITERS   evaluations spent on each root, int32
 *   EIG_DBG_W            the Q-basis eigenvector matrix, n-by-n doubles
 * Errors: EIG_EINVAL (unknown `what`, dst NULL or too small). */
enum {
  EIG_DBG_U = 1,
  EIG_DBG_POLE_COUNT = 2,
  EIG_DBG_SEG_START = 3,
  EIG_DBG_REDUCED_D = 4,
  EIG_DBG_REDUCED_ROW = 5,
  EIG_DBG_ROOT_ORIGIN = 6,
  EIG_DBG_ROOT_TAU = 7,
  EIG_DBG_ROOT_ITERS = 8,
  EIG_DBG_W = 9
};
int eig_debug_fetch(eig_state_t s, int32_t what, void *dst, int64_t bytes, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* EIGUPD_H */
