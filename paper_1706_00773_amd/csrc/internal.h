// internal.h -- shared declarations of the HIP translation units of libeigupd.
//
// Data layout in device memory (n = order, K = compile-time rank bound):
//   lam[2], Q[2]     two resident copies of (lambda, Q); an update reads one and
//                    writes the other, the commit flips which one is current
//   U                Q^T K, n rows of k doubles (row j = u_j, contiguous)
//   reduced problem  rd (poles), ru (rows, k doubles each), rrow (original row
//                    of each reduced row), rmap (original row -> reduced row or -1)
//   segments         distinct poles: seg_start (first reduced row), seg_r (rows)
//   deflated         dval (eigenvalue), drow (row of its unit vector)
//   roots            root_o (origin segment), root_tau (offset), root_c (k doubles:
//                    null vector scaled so that the eigenvector has unit norm)
//   colparam         per output column: origin pole, tau, signed c, or a unit row
//   W                n-by-n column-major eigenvectors in the Q basis
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "eigupd.h"

namespace eigupd {

constexpr int KMAX = 8;

// Deferred error bits (DevState::status)
constexpr int ST_NONFINITE = 1;
constexpr int ST_NOCONV = 2;
constexpr int ST_INTERNAL = 4;
constexpr int ST_CHECK = 8;  // a check of EIG_DEBUG_CHECKS failed

// The EIG_* status of a set of deferred error bits (the first kind wins).
__host__ __device__ inline int status_code(int bits) {
  if (bits & ST_NONFINITE) return EIG_ENONFINITE;
  if (bits & ST_NOCONV) return EIG_ENOCONV;
  if (bits & ST_CHECK) return EIG_ECHECK;
  if (bits) return EIG_EDEVICE;
  return EIG_OK;
}

// Deflation thresholds, relative to ahat = max|lambda| + ||U||_F^2 (>= ||A'||_2):
// a row u_j is dropped when ||u_j|| ||U||_F <= TAU_ROW * ahat; neighbouring poles
// closer than TAU_GAP * ahat are merged into one group.
constexpr double TAU_ROW = 1e-12;
constexpr double TAU_GAP = 8.0 * 1.1102230246251565e-16;

// Default iteration cap per root (count and Newton evaluations together);
// eig_state_set(EIG_KNOB_MAX_EVALS) changes it per state.
constexpr int MAX_EVALS = 160;

// Column chunks of the FP64 residual K - Q U0 in the reduced-precision modes.
constexpr int LP_RESID_CHUNKS = 16;

struct DevState {   // persistent for the life of a state
  int32_t status;   // sticky error bits
  int32_t pad;
  long long gen;    // committed updates since upload
};

struct DevInfo {    // written by the kernels of one update
  int32_t n_d, n_s, n_defl, n_groups;
  int32_t p, q, k, n_nt;
  double ahat, fro2, lower, upper, bwd;
  int32_t it_min, it_max;
  long long it_sum;
  int32_t alpha_bad;   // residue location: a residue too small to trust its sign
  int32_t loc_alpha;   // 1: the pole counts came from the residue signs
  int32_t r_lo, r_hi;  // roots of the reduced problem to solve (all: 0, n_d)
  int32_t e_lo, e_hi;  // deflated eigenvalues to keep (all: 0, n_defl)
  int32_t root_next;   // root solver: roots handed out so far (from r_lo)
  int32_t pad_;
};

struct ColParam {   // one output column of W
  double d_o;       // origin pole value (root columns)
  double tau;       // offset of the root from d_o
  double c[KMAX];   // signed, scaled null vector
  int32_t drow;     // >= 0: unit vector e_drow (deflated column); -1: root column
  int32_t pad;
};

struct Work {
  int n, k, ldk, sig_pos_mask;  // bit c of sig_pos_mask set <=> sigma_c = +1
  int ncols;                    // columns of W built (n, or the size of a subset)
  int ldq;                      // leading dimension of Q_in as read by U = Q^T K
  int max_evals;                // evaluations per root before ST_NOCONV is raised
  int pad2_;
  const double* lam_in;
  const double* Q_in;
  double* lam_out;
  double* Q_out;
  double* lam_fin;  // where the merged eigenvalues go: lam_out, or a values-only buffer
  const double* K;
  double* U;
  // deflation
  int* tiny;        // n   row flags
  int* nt_list;     // n   non-tiny rows in order
  int* grp_id;      // n   group of each non-tiny position
  int* g_first;     // n   first non-tiny position of each group
  int* g_m;         // n   group size
  int* g_r;         // n   kept rows of each group
  int* g_h;         // n   reflectors of each group
  double* g_val;    // n   pole value of each group
  double* hv;       // n*KMAX reflector vectors (by non-tiny position)
  double* hbeta;    // n*KMAX reflector scalars (by group)
  double* urot;     // n*KMAX rotated rows (by non-tiny position)
  int* mg_list;     // n   groups with two or more rows
  double* rd;       // n
  double* ru;       // n*KMAX
  int* rrow;        // n
  int* rmap;        // n
  int* row_seg;     // n   segment of each reduced row
  int* seg_start;   // n+1
  int* seg_r;       // n
  double* dval;     // n
  int* drow;        // n
  // location and roots
  int* nu;          // n   pole counts
  int* root_t;      // n   interval of each root
  int* root_clo;    // n   count at the interval's left end
  int* root_chi;    // n   count at the interval's right end
  int* root_o;      // n   origin segment
  double* root_tau; // n
  double* root_tv;  // n   offset at which the root's null vector was formed
  double* root_c;   // n*KMAX
  int* root_it;     // n
  double* xs;       // n   absolute root values (monotone)
  ColParam* colp;   // n
  double* W;        // n*n
  // reduced-precision modes
  double* lp_part;  // LP_RESID_CHUNKS*n*KMAX partial products of Q U0
  double* lp_resid; // n*KMAX residual K - Q U0 (column-major, leading dimension n)
  DevState* st;
  DevInfo* info;
};

// A grouped launch runs one kernel over several instances of the same rank k:
// block b of the grid belongs to the instance i with prefix[i] <= b <
// prefix[i + 1] and is that instance's block b - prefix[i].
struct Group {
  const Work* works;  // ninst descriptors in device memory
  const int* prefix;  // ninst + 1 block offsets in device memory
  int ninst;
};

__device__ __forceinline__ int group_instance(const Group& g, int b) {
  int lo = 0, hi = g.ninst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (g.prefix[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// switch over the compile-time rank: EIGUPD_SWITCH_K(k, fn, args...) returns
// fn<k>(args...) for k = 1..KMAX
#define EIGUPD_SWITCH_K(kval, fn, ...)            \
  switch (kval) {                                 \
    case 1: return fn<1>(__VA_ARGS__);            \
    case 2: return fn<2>(__VA_ARGS__);            \
    case 3: return fn<3>(__VA_ARGS__);            \
    case 4: return fn<4>(__VA_ARGS__);            \
    case 5: return fn<5>(__VA_ARGS__);            \
    case 6: return fn<6>(__VA_ARGS__);            \
    case 7: return fn<7>(__VA_ARGS__);            \
    case 8: return fn<8>(__VA_ARGS__);            \
    default: return hipErrorInvalidValue;         \
  }

// One instance of the grouped FP64 product C = A B (all n x n, leading
// dimension n); vec: 16-byte accesses allowed (n even, aligned pointers).
struct GemmDesc {
  const double* A;
  const double* B;
  double* C;
  const int32_t* status;
  int n;
  int vec;
};

// One product C (+)= A B of a general shape, column-major, built on the device;
// tiles_m = ceil(M / tile side); vec: 16-byte accesses allowed.
struct GemmDescG {
  const double* A;
  const double* B;
  double* C;
  int M, N, K, lda, ldb, ldc, vec, tiles_m;
};

// C = sum_i A_i B_i over up to GSEG operand pairs (all M rows, N columns;
// A_i is M x K_i, B_i is K_i x N, column-major), built on the device; send[i] =
// k-slices (of 16) of pairs 0..i together; vec: 16-byte accesses allowed for
// every pair and C.
constexpr int GSEG = 6;
struct GemmSegDesc {
  const double* A[GSEG];
  const double* B[GSEG];
  double* C;
  int lda[GSEG], ldb[GSEG], K[GSEG], send[GSEG];
  int M, N, ldc, vec, tiles_m, nseg;
};

// Q' = Q W with the far blocks of W from Chebyshev expansions (farfield.hip):
// buffers of one state, laid out by ff_layout in ff_bytes(n, k) bytes.
struct FarField {
  int n, k, nb, nr;     // column blocks of 256 columns, row blocks of rb rows
  int rb, pr, pc, pad;  // row block size; nodes per row / column interval
  double etar, etac;    // far: distance >= etac column width and >= etar row width
  double* M;      // (k n) x (nr pr) expansions of the row blocks
  double* L;      // (k n) x (nb pc) expansions at the column blocks
  double* T;      // (nr pr) x (nb pc) interaction matrix
  double* B;      // row-block weights, b_h x k pr each
  double* Phi;    // k pc x n column weights
  double* ivr;    // 2 per row block: pole interval
  double* ivc;    // 2 per column block: column-point interval
  double* xn;     // nb pc column-block nodes
  double* yn;     // nr pr row-block nodes
  GemmDescG* desc;    // nr: P2M
  GemmSegDesc* seg;   // nb: near rows + L2P of each column block, in launch order
  int* prefix;        // (nr + 1) + (nb + 1) tile offsets: P2M, segmented products
  int* near;      // 2 nb: first and last row block of each band
  int* extra;     // 2 (GSEG - 2) nb: further near row-block ranges [lo, hi] (lo < 0: none)
  int* flags;     // [0] far path skipped, [1] dense path skipped
};
// Rows [ff_row_begin, ff_row_end) of row block h (the last block takes the rest).
__host__ __device__ inline int ff_row_begin(const FarField& f, int h) { return h * f.rb; }
__host__ __device__ inline int ff_row_end(const FarField& f, int h) {
  return h + 1 >= f.nr ? f.n : (h + 1) * f.rb;
}
// Row block h is multiplied exactly for column block I (band or further range).
__device__ inline bool ff_near(const FarField& f, int I, int h) {
  bool hit = h >= f.near[2 * I] && h <= f.near[2 * I + 1];
  for (int r = 0; r < GSEG - 2; ++r) {
    const int lo = f.extra[2 * (I * (GSEG - 2) + r)], hi = f.extra[2 * (I * (GSEG - 2) + r) + 1];
    hit = hit || (h >= lo && h <= hi);
  }
  return hit;
}
bool ff_eligible(int n, int k);
int ff_blocks(int n);
size_t ff_bytes(int n, int k);
size_t ff_bytes_max(int n);  // the most ff_bytes(n, k) over every rank
FarField ff_layout(void* base, int n, int k);
// The plan (intervals, near bands, path decision); needs finalize to have run.
hipError_t launch_ff_plan(const Work& w, const FarField& f, hipStream_t s);
// W on the blocks the far-field product reads (all of W if the plan fell back).
hipError_t launch_wbuild_ff(const Work& w, const FarField& f, hipStream_t s);
// Both product paths (one of them exits at once): Q_out = Q_in W.  Needs the
// plan and W (launch_wbuild_ff, then group reflectors) to have run.
hipError_t launch_qw_farfield(const Work& w, const FarField& f, hipStream_t s);

// EIG_DEBUG_CHECKS (checks.hip): eigenvalue order, Courant-Weyl windows and the
// trace always; 8 sampled columns of W (residual, Gram) when check_w; the same
// columns of Q_out (Gram within tol_q) when check_q.  Raises ST_CHECK.
hipError_t launch_debug_checks(const Work& w, bool check_w, bool check_q, double tol_q,
                               hipStream_t s);

// Launchers (stream-ordered, no allocation).
hipError_t launch_qtk(const Work& w, hipStream_t s);
hipError_t launch_deflate(const Work& w, hipStream_t s);
hipError_t launch_polecount(const Work& w, hipStream_t s);
// Rank 2 only: pole counts from the signs of the residues alpha_s (eq. (2)) and
// the Courant-Weyl bounds; leaves info->loc_alpha = 0 (and the pole-count
// kernel then runs) when a residue is too small for its sign to be certain.
hipError_t launch_alpha_locate(const Work& w, hipStream_t s);
hipError_t launch_locate(const Work& w, hipStream_t s);
// Subset of the spectrum: sets info->r_lo/r_hi to the roots of the reduced
// problem in [a, b) and info->e_lo/e_hi to the deflated eigenvalues in [a, b)
// (after deflate, polecount and locate).
hipError_t launch_interval_count(const Work& w, double a, double b, hipStream_t s);
// nroots >= 0: grid for that many roots (starting at info->r_lo); default all n
hipError_t launch_rootsolve(const Work& w, hipStream_t s, int nroots = -1);
hipError_t launch_finalize(const Work& w, hipStream_t s);
hipError_t launch_wbuild(const Work& w, hipStream_t s);
hipError_t launch_group_reflect(const Work& w, hipStream_t s);
hipError_t launch_commit(const Work& w, hipStream_t s);
// First-order perturbation estimate (eq. (11)): lam_out and W = I + C from U.
hipError_t launch_perturb_w(const Work& w, double* lam_out, hipStream_t s);
// C = A * B, column-major, FP64 MFMA.  Skipped on the device when *status != 0.
hipError_t launch_dgemm(int M, int N, int Kd, const double* A, int lda, const double* B, int ldb,
                        double* C, int ldc, const int32_t* status, hipStream_t s);
// Segmented products from ninst device-built descriptors (tiles as below).
// V = Q W for m <= 128 columns (subset.hip): split-k partial sums in `part`
// (skinny_workspace bytes), then their ordered sum; needs n and ldq even and Q
// 16-byte aligned (skinny_applies).
size_t skinny_workspace(int n, int m);
bool skinny_applies(int n, int m, const double* Q, int ldq);
hipError_t launch_skinny_qw(int n, int m, const double* Q, int ldq, const double* W, int ldw,
                            double* V, int ldv, double* part, const int32_t* status,
                            hipStream_t s);
hipError_t launch_dgemm_seg(const GemmSegDesc* d, const int* prefix, int ninst, int blocks,
                            const int32_t* skip, hipStream_t s);
// Products from ninst device-built descriptors (acc: C += A B) on bt x bt tiles
// (128, or 64 without acc; tiles_m = ceil(M / bt)); block b of the grid is tile
// b - prefix[i] of instance i; skipped on the device when *skip != 0.
hipError_t launch_dgemm_desc(bool acc, int bt, const GemmDescG* d, const int* prefix, int ninst,
                             int blocks, const int32_t* skip, hipStream_t s);
// Grouped launches over `ninst` instances of one rank k (blocks = total blocks,
// Group.prefix built from the per-instance counts below).
int qtk_blocks(int n, int k);
int root_blocks(int n);   // polecount / rootvec blocks of an instance
int solve_blocks(int n, int k);  // rootsolve blocks of an instance
int wbuild_blocks(int n);
int reflect_blocks(int n);
int gemm_tiles(int n, int bt);
hipError_t launch_qtk_group(int k, const Group& g, int blocks, hipStream_t s);
hipError_t launch_deflate_group(int k, const Work* works, int ninst, hipStream_t s);
hipError_t launch_polecount_group(int k, const Group& g, int blocks, hipStream_t s);
hipError_t launch_locate_group(const Work* works, int ninst, hipStream_t s);
// persistent_grid > 0: that many blocks draw (instance, root block) items from
// *queue (reset on the stream first); 0: one block per item.
// Secular Sturm chain (chain.hip): residues, found-zero deflation, level 1 and
// the serial build into ws (chain_ws_doubles(n_d) doubles); then the counts.
size_t chain_ws_doubles(int n_d);
hipError_t launch_chain(const Work& w, int n_d, const double* xi, int n_xi, double* ws, int* bad,
                        hipStream_t s);
hipError_t launch_chain_count(const Work& w, int n_d, const double* xi, int n_xi,
                              const double* ws, int levels, const double* x, int n_x,
                              int64_t* counts, hipStream_t s);
hipError_t launch_rootsolve_group(int k, const Group& gs, int solve_blocks, const Group& gv,
                                  int vec_blocks, int persistent_grid, int* queue,
                                  hipStream_t s);
hipError_t launch_finalize_group(int k, const Work* works, int ninst, hipStream_t s);
hipError_t launch_wbuild_group(int k, const Group& g, int blocks, hipStream_t s);
hipError_t launch_reflect_group(int k, const Group& g, int blocks, hipStream_t s);
hipError_t launch_commit_group(const Work* works, int ninst, hipStream_t s);
// bt = 128 or 64 (tile side); blocks = sum of gemm_tiles(n_i, bt)
hipError_t launch_dgemm_group(int bt, const GemmDesc* d, const int* prefix, int ninst, int blocks,
                              hipStream_t s);

// Reduced-precision variants (prec = EIG_GEMM_FP32_CORR or EIG_GEMM_BF16X3_CORR):
// U = Q^T K with the FP64 residual correction, and C = A * B on the matrix cores.
hipError_t launch_qtk_lp(const Work& w, int prec, hipStream_t s);
// Q_out = Q_in W: splits W and Q into the slice planes qplanes / wplanes (each
// lp_plane_bytes(prec, n) bytes), then runs the matrix-core product.
size_t lp_plane_bytes(int prec, int n);
hipError_t launch_gemm_lp(const Work& w, int prec, void* qplanes, void* wplanes, hipStream_t s);

}  // namespace eigupd
