// api.hip -- the C ABI of libeigupd (declared in include/eigupd.h): state
// management, argument checks and the stream-ordered launch sequence of one
// rank-k update.  All device memory is allocated once, in eig_state_create.
#include <math.h>

#include <cmath>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "eigupd.h"
#include "internal.h"
#include "state.h"
#include "trace.h"

using namespace eigupd;


namespace {

struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = (hipSetDevice(dev) == hipSuccess);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// Lays out every buffer of a state of order n inside `base` (nullptr: sizing pass).
size_t carve(eig_state_s* s, void* base) {
  const size_t n = (size_t)s->n;
  Carver c(base);
  s->lam[0] = c.take<double>(n);
  s->lam[1] = c.take<double>(n);
  s->lam_vo = c.take<double>(n);
  s->lam_x = c.take<double>(n);
  Work& w = s->w;
  if (s->lean) {
    // Q and W buffers are lent per update by the owner of the state
    s->Q[0] = s->Q[1] = nullptr;
    w.W = nullptr;
  } else {
    s->Q[0] = c.take<double>(n * n);
    s->Q[1] = c.take<double>(n * n);
    w.W = c.take<double>(n * n);
  }
  s->Kbuf = c.take<double>(n * EIG_KMAX_GENERIC);
  c.off = carve_workspace(w, n, static_cast<char*>(base), c.off);
  w.lp_part = c.take<double>((size_t)LP_RESID_CHUNKS * n * KMAX);
  w.lp_resid = c.take<double>(n * KMAX);
  return c.off + 256;
}

}  // namespace

namespace eigupd {

size_t carve_workspace(Work& w, size_t n, char* base, size_t off) {
  Carver c(base);
  c.off = off;
  w.U = c.take<double>(n * KMAX);
  w.tiny = c.take<int>(n);
  w.nt_list = c.take<int>(n);
  w.grp_id = c.take<int>(n);
  w.g_first = c.take<int>(n);
  w.g_m = c.take<int>(n);
  w.g_r = c.take<int>(n);
  w.g_h = c.take<int>(n);
  w.g_val = c.take<double>(n);
  w.hv = c.take<double>(n * KMAX);
  w.hbeta = c.take<double>(n * KMAX);
  w.urot = c.take<double>(n * KMAX);
  w.mg_list = c.take<int>(n);
  w.rd = c.take<double>(n);
  w.ru = c.take<double>(n * KMAX);
  w.rrow = c.take<int>(n);
  w.rmap = c.take<int>(n);
  w.row_seg = c.take<int>(n);
  w.seg_start = c.take<int>(n + 1);
  w.seg_r = c.take<int>(n);
  w.dval = c.take<double>(n);
  w.drow = c.take<int>(n);
  w.nu = c.take<int>(n);
  w.root_t = c.take<int>(n);
  w.root_clo = c.take<int>(n);
  w.root_chi = c.take<int>(n);
  w.root_o = c.take<int>(n);
  w.root_tau = c.take<double>(n);
  w.root_tv = c.take<double>(n);
  w.root_c = c.take<double>(n * KMAX);
  w.root_it = c.take<int>(n);
  w.xs = c.take<double>(n);
  w.colp = c.take<ColParam>(n);
  w.st = c.take<DevState>(1);
  w.info = c.take<DevInfo>(1);
  return c.off;
}

}  // namespace eigupd

namespace {

int status_from_bits(int bits) { return status_code(bits); }

#define HIPCHK(x)                                   \
  do {                                              \
    if ((x) != hipSuccess) return EIG_EDEVICE;      \
  } while (0)

// Writes the device status `ds` with its sticky bits cleared, and waits until
// the write has landed: a host-to-device hipMemcpy may return before its DMA
// ends, and a later update on a non-blocking stream would then still see the
// old bits.
hipError_t clear_status(DevState* dst, DevState ds, hipStream_t st) {
  ds.status = 0;
  hipError_t e = hipMemcpyAsync(dst, &ds, sizeof(ds), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e;
}

// Enqueues one update of rank w.k <= KMAX with the buffers in w: U = Q^T K,
// deflation, location, roots, the merged eigenvalues, and (unless
// values_only) W and Q_out = Q_in W; then the debug checks if asked.  Nothing
// is committed.  mark(e) is called between the phases (e = 1..6, as in
// eig_info.ms).
template <typename Mark>
int enqueue_part(eig_state_s* s, const Work& w, int prec, bool farfield, bool residues,
                 bool checks, bool values_only, hipStream_t st, Mark&& mark) {
  const int n = (int)s->n;
  {
    TraceRange r("eig.qtk");
    if (prec == EIG_GEMM_FP64)
      HIPCHK(launch_qtk(w, st));
    else
      HIPCHK(launch_qtk_lp(w, prec, st));
  }
  HIPCHK(mark(1));
  {
    TraceRange r("eig.deflate");
    HIPCHK(launch_deflate(w, st));
  }
  HIPCHK(mark(2));
  {
    TraceRange r("eig.locate");
    if (residues && w.k == 2) HIPCHK(launch_alpha_locate(w, st));
    HIPCHK(launch_polecount(w, st));
    HIPCHK(launch_locate(w, st));
  }
  HIPCHK(mark(3));
  {
    TraceRange r("eig.roots");
    HIPCHK(launch_rootsolve(w, st));
  }
  HIPCHK(mark(4));
  {
    TraceRange r("eig.merge");
    HIPCHK(launch_finalize(w, st));
  }
  if (values_only) {
    if (checks) {
      TraceRange r("eig.checks");
      HIPCHK(launch_debug_checks(w, false, false, 0.0, st));
    }
    HIPCHK(mark(5));
    HIPCHK(mark(6));
    return EIG_OK;
  }
  const bool ff = farfield && ff_eligible(n, w.k);
  const FarField f = ff ? ff_layout(s->ff_block, n, w.k) : FarField{};
  {
    TraceRange r("eig.w");
    if (ff) {
      HIPCHK(launch_ff_plan(w, f, st));
      HIPCHK(launch_wbuild_ff(w, f, st));
    } else {
      HIPCHK(launch_wbuild(w, st));
    }
    HIPCHK(launch_group_reflect(w, st));
  }
  HIPCHK(mark(5));
  {
    TraceRange r(ff ? "eig.qw_farfield" : "eig.qw");
    if (ff)
      HIPCHK(launch_qw_farfield(w, f, st));
    else if (prec == EIG_GEMM_FP64)
      HIPCHK(launch_dgemm(n, n, n, w.Q_in, n, w.W, n, w.Q_out, n, &w.st->status, st));
    else
      HIPCHK(launch_gemm_lp(w, prec, s->lp_block,
                            static_cast<char*>(s->lp_block) + s->lp_bytes / 2, st));
  }
  HIPCHK(mark(6));
  if (checks) {
    TraceRange r("eig.checks");
    // W is whole unless the far-field product formed only its near blocks; the
    // reduced products' bound on Q'^T Q' - I is 2 sqrt(n) 4e-6
    const double tol_q = (prec == EIG_GEMM_FP64) ? 1e-9 : 8e-6 * std::sqrt((double)n);
    HIPCHK(launch_debug_checks(w, !ff, true, tol_q, st));
  }
  return EIG_OK;
}

}  // namespace

extern "C" {

const char* eig_status_str(int status) {
  switch (status) {
    case EIG_OK: return "ok";
    case EIG_EINVAL: return "invalid argument";
    case EIG_ENOMEM: return "out of device memory";
    case EIG_EDEVICE: return "HIP device or runtime error";
    case EIG_ENOCONV: return "a secular root did not converge";
    case EIG_ENOTSORTED: return "eigenvalues not ascending";
    case EIG_EUNSUPPORTED: return "unsupported rank or mode";
    case EIG_EDEPENDENCY: return "a predecessor update failed";
    case EIG_ESTATE: return "state has no decomposition (upload first)";
    case EIG_ENONFINITE: return "non-finite value in the input";
    case EIG_ECHECK: return "a check of EIG_DEBUG_CHECKS failed";
    default: return "unknown status";
  }
}

int eig_state_create(eig_state_t* out, int64_t n, int32_t device) {
  return eigupd::state_create(out, n, device, false);
}

}  // extern "C"

namespace eigupd {

int state_create(eig_state_t* out, int64_t n, int32_t device, bool lean) {
  if (!out || n < 1 || n > (int64_t)1 << 30) return EIG_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return EIG_EDEVICE;
  DeviceGuard g(device);
  if (!g.ok) return EIG_EDEVICE;
  eig_state_s* s = new (std::nothrow) eig_state_s();
  if (!s) return EIG_ENOMEM;
  s->device = device;
  s->n = n;
  s->lean = lean;
  s->w.n = (int)n;
  s->w.ncols = (int)n;
  s->w.ldq = (int)n;
  s->w.max_evals = MAX_EVALS;
  const size_t bytes = carve(s, nullptr);
  void* block = nullptr;
  if (hipMalloc(&block, bytes) != hipSuccess) {
    delete s;
    (void)hipGetLastError();
    return EIG_ENOMEM;
  }
  s->block = block;
  s->block_bytes = bytes;
  carve(s, block);
  for (auto& e : s->ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      for (auto& f : s->ev)
        if (f) (void)hipEventDestroy(f);
      (void)hipFree(block);
      delete s;
      return EIG_EDEVICE;
    }
  }
  DevState z{};
  if (hipMemcpy(s->w.st, &z, sizeof(z), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(block);
    delete s;
    return EIG_EDEVICE;
  }
  *out = s;
  return EIG_OK;
}

}  // namespace eigupd

extern "C" {

int eig_state_destroy(eig_state_t s) {
  if (!s) return EIG_EINVAL;
  {
    DeviceGuard g(s->device);
    (void)hipDeviceSynchronize();
    for (auto& e : s->ev)
      if (e) (void)hipEventDestroy(e);
    if (s->block) (void)hipFree(s->block);
    if (s->lp_block) (void)hipFree(s->lp_block);
    if (s->ff_block) (void)hipFree(s->ff_block);
    if (s->Q_x) (void)hipFree(s->Q_x);
  }
  delete s;
  return EIG_OK;
}

int eig_state_set(eig_state_t s, int32_t knob, int64_t value) {
  if (!s) return EIG_EINVAL;
  switch (knob) {
    case EIG_KNOB_MAX_EVALS:
      if (value < 1 || value > 1000000) return EIG_EINVAL;
      s->w.max_evals = (int)value;
      return EIG_OK;
    default:
      return EIG_EINVAL;
  }
}

int eig_state_upload(eig_state_t s, const double* lambda, const double* Q, int64_t ldq,
                     int32_t ptrs_on_device, void* hip_stream) {
  TraceRange trace("eig_state_upload");
  if (!s || !lambda || !Q || ldq < s->n || s->lean) return EIG_EINVAL;
  DeviceGuard g(s->device);
  if (!g.ok) return EIG_EDEVICE;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const size_t n = (size_t)s->n;
  std::vector<double> h(n);
  const hipMemcpyKind kind = ptrs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (ptrs_on_device) {
    HIPCHK(hipMemcpyAsync(h.data(), lambda, n * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  } else {
    memcpy(h.data(), lambda, n * sizeof(double));
  }
  for (size_t j = 0; j < n; ++j) {
    if (!isfinite(h[j])) return EIG_ENOTSORTED;
    if (j > 0 && !(h[j] >= h[j - 1])) return EIG_ENOTSORTED;
  }
  HIPCHK(hipMemcpyAsync(s->lam[0], h.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpy2DAsync(s->Q[0], n * sizeof(double), Q, (size_t)ldq * sizeof(double),
                          n * sizeof(double), n, kind, st));
  DevState z{};
  HIPCHK(hipMemcpyAsync(s->w.st, &z, sizeof(z), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  s->enq_gen = 0;
  s->uploaded = true;
  s->last_vo = false;
  return EIG_OK;
}

int eig_update_rankk(eig_state_t s, int64_t k, const double* K, int64_t ldk, const int8_t* sigma,
                     uint32_t mode, void* hip_stream) {
  TraceRange trace("eig_update_rankk");
  if (!s || !K || !sigma || k < 1 || ldk < s->n || s->lean) return EIG_EINVAL;
  if (k > EIG_KMAX_GENERIC) return EIG_EUNSUPPORTED;
  if (k > s->n || ldk > INT32_MAX) return EIG_EINVAL;
  const uint32_t known = EIG_GEMM_MASK | EIG_VALUES_ONLY | EIG_HOST_INPUT | EIG_PHASE_TIMING |
                         EIG_LOCATE_RESIDUES | EIG_QW_FARFIELD | EIG_DEBUG_CHECKS;
  if (mode & ~known) return EIG_EUNSUPPORTED;
  const int prec = (int)(mode & EIG_GEMM_MASK);
  if (prec != EIG_GEMM_FP64 && prec != EIG_GEMM_FP32_CORR && prec != EIG_GEMM_BF16X3_CORR)
    return EIG_EUNSUPPORTED;
  int npos = 0;
  for (int64_t c = 0; c < k; ++c) {
    if (sigma[c] == 1)
      ++npos;
    else if (sigma[c] != -1)
      return EIG_EINVAL;
  }
  if (!s->uploaded) return EIG_ESTATE;
  DeviceGuard g(s->device);
  if (!g.ok) return EIG_EDEVICE;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const size_t n = (size_t)s->n;
  const bool vo = (mode & EIG_VALUES_ONLY) != 0;
  // ranks above EIG_KMAX: ceil(k / EIG_KMAX) parts of nearly equal rank, applied in turn
  const int parts = (int)((k + EIG_KMAX - 1) / EIG_KMAX);
  const int part_k = (int)((k + parts - 1) / parts);  // the largest part
  const double* Kd = K;
  int64_t ldkd = ldk;
  if (mode & EIG_HOST_INPUT) {
    HIPCHK(hipMemcpy2DAsync(s->Kbuf, n * sizeof(double), K, (size_t)ldk * sizeof(double),
                            n * sizeof(double), (size_t)k, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    Kd = s->Kbuf;
    ldkd = (int64_t)n;
  }
  // buffers allocated on first use: slice planes of the reduced modes, the
  // far-field product's expansions, and a second Q for the chained parts
  auto grow = [&](void** blk, size_t* have, size_t need) -> int {
    if (*have >= need) return EIG_OK;
    if (*blk) {
      HIPCHK(hipStreamSynchronize(st));
      HIPCHK(hipDeviceSynchronize());
      (void)hipFree(*blk);
      *blk = nullptr;
      *have = 0;
    }
    if (hipMalloc(blk, need) != hipSuccess) {
      (void)hipGetLastError();
      *blk = nullptr;
      return EIG_ENOMEM;
    }
    *have = need;
    return EIG_OK;
  };
  const bool any_product = !vo || parts > 1;
  if (prec != EIG_GEMM_FP64 && any_product) {
    const int rc = grow(&s->lp_block, &s->lp_bytes, 2 * lp_plane_bytes(prec, (int)n));
    if (rc != EIG_OK) return rc;
  }
  const bool farfield = (mode & EIG_QW_FARFIELD) && prec == EIG_GEMM_FP64 && any_product &&
                        ff_eligible((int)n, part_k);
  if (farfield) {
    // the parts' ranks differ by at most one; the buffers depend on the rank
    // through the row-block size too, so take the larger need of the two
    const size_t ffb = std::max(ff_bytes((int)n, part_k), ff_bytes((int)n, (int)(k / parts)));
    const int rc = grow(&s->ff_block, &s->ff_bytes, ffb);
    if (rc != EIG_OK) return rc;
  }
  if (parts > 1 && !s->Q_x) {
    void* q = nullptr;
    size_t have = 0;
    const int rc = grow(&q, &have, n * n * sizeof(double));
    if (rc != EIG_OK) return rc;
    s->Q_x = static_cast<double*>(q);
  }
  const bool timed = (mode & EIG_PHASE_TIMING) != 0;
  const bool checks = (mode & EIG_DEBUG_CHECKS) != 0;
  const int cur = (int)(s->enq_gen & 1);
  double* lam_final = vo ? s->lam_vo : s->lam[cur ^ 1];
  Work w = s->w;
  if (timed) HIPCHK(hipEventRecord(s->ev[0], st));
  int c0 = 0;
  for (int i = 0; i < parts; ++i) {
    const int kc = (int)(k / parts) + (i < (int)(k % parts) ? 1 : 0);
    const bool last = (i == parts - 1);
    // the last part writes the state's other buffers, the one before it the
    // spare ones, and so on back: no part writes what it reads, and the
    // committed (lambda, Q) is read but never written
    const bool to_final = ((parts - 1 - i) % 2) == 0;
    int mask = 0;
    for (int c = 0; c < kc; ++c) mask |= (sigma[c0 + c] == 1) ? (1 << c) : 0;
    const double* lam_in = (i == 0) ? s->lam[cur] : w.lam_fin;
    const double* Q_in = (i == 0) ? s->Q[cur] : w.Q_out;
    w = s->w;
    w.k = kc;
    w.sig_pos_mask = mask;
    w.K = Kd + (size_t)c0 * ldkd;
    w.ldk = (int)ldkd;
    w.lam_in = lam_in;
    w.Q_in = Q_in;
    w.lam_out = to_final ? s->lam[cur ^ 1] : s->lam_x;
    w.lam_fin = to_final ? lam_final : s->lam_x;
    w.Q_out = to_final ? s->Q[cur ^ 1] : s->Q_x;
    auto mark = [&](int e) -> hipError_t {
      return (timed && last && e > 0) ? hipEventRecord(s->ev[e], st) : hipSuccess;
    };
    TraceRange part_range(parts > 1 ? "eig.part" : "eig.update");
    const int rc = enqueue_part(s, w, prec, farfield, (mode & EIG_LOCATE_RESIDUES) != 0, checks,
                                vo && last, st, mark);
    if (rc != EIG_OK) return rc;
    c0 += kc;
  }
  s->last_k = (int)k;
  s->last_p = npos;
  s->last_q = (int)k - npos;
  s->timed = timed;
  if (!vo) HIPCHK(launch_commit(w, st));
  if (timed) {
    HIPCHK(hipEventRecord(s->ev[7], st));
    HIPCHK(hipEventRecord(s->ev[8], st));
  }
  if (!vo) s->enq_gen += 1;
  s->last_vo = vo;
  return EIG_OK;
}

int eig_update_interval(eig_state_t s, int64_t k, const double* K, int64_t ldk,
                        const int8_t* sigma, double a, double b, uint32_t mode,
                        double* lambda_out, double* V_out, int64_t ldv, int64_t m_max,
                        int64_t* m_out, void* hip_stream) {
  TraceRange trace("eig_update_interval");
  if (!s || !K || !sigma || !m_out || k < 1 || ldk < s->n || s->lean) return EIG_EINVAL;
  *m_out = 0;
  if (k > EIG_KMAX) return EIG_EUNSUPPORTED;
  if (k > s->n || std::isnan(a) || std::isnan(b) || !(a <= b) || m_max < 0) return EIG_EINVAL;
  const uint32_t known = EIG_VALUES_ONLY | EIG_HOST_INPUT | EIG_LOCATE_RESIDUES;
  if (mode & ~known) return EIG_EUNSUPPORTED;
  const bool vo = (mode & EIG_VALUES_ONLY) != 0;
  if (m_max > 0 && !lambda_out) return EIG_EINVAL;
  if (!vo && m_max > 0 && (!V_out || ldv < s->n)) return EIG_EINVAL;
  int mask = 0;
  for (int64_t c = 0; c < k; ++c) {
    if (sigma[c] == 1)
      mask |= 1 << c;
    else if (sigma[c] != -1)
      return EIG_EINVAL;
  }
  if (!s->uploaded) return EIG_ESTATE;
  DeviceGuard g(s->device);
  if (!g.ok) return EIG_EDEVICE;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const size_t n = (size_t)s->n;
  const double* Kd = K;
  int64_t ldkd = ldk;
  if (mode & EIG_HOST_INPUT) {
    HIPCHK(hipMemcpy2DAsync(s->Kbuf, n * sizeof(double), K, (size_t)ldk * sizeof(double),
                            n * sizeof(double), (size_t)k, hipMemcpyHostToDevice, st));
    Kd = s->Kbuf;
    ldkd = (int64_t)n;
  }
  Work w = make_work(s, (int)k, Kd, (int)ldkd, mask, true);
  // phase 1: U, deflation, location, and the roots that fall in [a, b)
  HIPCHK(launch_qtk(w, st));
  HIPCHK(launch_deflate(w, st));
  if ((mode & EIG_LOCATE_RESIDUES) && k == 2) HIPCHK(launch_alpha_locate(w, st));
  HIPCHK(launch_polecount(w, st));
  HIPCHK(launch_locate(w, st));
  HIPCHK(launch_interval_count(w, a, b, st));
  HIPCHK(hipStreamSynchronize(st));
  DevState ds;
  DevInfo di;
  HIPCHK(hipMemcpy(&ds, s->w.st, sizeof(ds), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(&di, s->w.info, sizeof(di), hipMemcpyDeviceToHost));
  auto device_error = [&]() -> int {
    // report a device error and clear it: the state keeps its committed pair
    if (clear_status(s->w.st, ds, st) != hipSuccess) return EIG_EDEVICE;
    return status_from_bits(ds.status);
  };
  if (ds.status != 0) return device_error();
  const int nr = di.r_hi - di.r_lo, ne = di.e_hi - di.e_lo;
  const int64_t m = (int64_t)nr + ne;
  *m_out = m;
  if (m > m_max) return EIG_EINVAL;
  s->last_k = (int)k;
  s->last_p = __builtin_popcount((unsigned)mask);
  s->last_q = (int)k - s->last_p;
  if (m == 0) return EIG_OK;
  // phase 2: those roots, their vectors, W (n x m) and V = Q W (2 n^2 m flops)
  w.lam_fin = lambda_out;
  w.ncols = (int)m;
  HIPCHK(launch_rootsolve(w, st, nr));
  HIPCHK(launch_finalize(w, st));
  if (!vo) {
    HIPCHK(launch_wbuild(w, st));
    HIPCHK(launch_group_reflect(w, st));
    // a few columns: the split-k product on the vector units, its partial sums
    // in the spare n x n buffer (nothing is committed here)
    if (skinny_applies((int)n, (int)m, w.Q_in, (int)n) &&
        skinny_workspace((int)n, (int)m) <= n * n * sizeof(double))
      HIPCHK(launch_skinny_qw((int)n, (int)m, w.Q_in, (int)n, w.W, (int)n, V_out, (int)ldv,
                              w.Q_out, &w.st->status, st));
    else
      HIPCHK(launch_dgemm((int)n, (int)m, (int)n, w.Q_in, (int)n, w.W, (int)n, V_out, (int)ldv,
                          &w.st->status, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipMemcpy(&ds, s->w.st, sizeof(ds), hipMemcpyDeviceToHost));
  if (ds.status != 0) return device_error();
  return EIG_OK;
}

int eig_sturm_chain(eig_state_t s, int64_t k, const double* K, int64_t ldk,
                    const int8_t* sigma, const double* xi, int64_t n_xi, const double* x,
                    int64_t n_x, int64_t* counts, double* c_out, int64_t c_max,
                    eig_chain_info* info, void* hip_stream) {
  TraceRange trace("eig_sturm_chain");
  if (!s || !K || !sigma || !info || k < 1 || ldk < s->n || s->lean) return EIG_EINVAL;
  if (n_xi < 0 || (n_xi > 0 && !xi) || n_x < 0 || (n_x > 0 && (!x || !counts)) || c_max < 0 ||
      (c_max > 0 && !c_out) || n_x > INT32_MAX)
    return EIG_EINVAL;
  if (k > EIG_KMAX) return EIG_EUNSUPPORTED;
  if (k > s->n) return EIG_EINVAL;
  int mask = 0;
  for (int64_t c = 0; c < k; ++c) {
    if (sigma[c] == 1)
      mask |= 1 << c;
    else if (sigma[c] != -1)
      return EIG_EINVAL;
  }
  if (!s->uploaded) return EIG_ESTATE;
  DeviceGuard g(s->device);
  if (!g.ok) return EIG_EDEVICE;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const size_t n = (size_t)s->n;
  Work w = make_work(s, (int)k, K, (int)ldk, mask, true);
  // U, deflation (the chain needs the reduced problem's simple poles)
  HIPCHK(launch_qtk(w, st));
  HIPCHK(launch_deflate(w, st));
  HIPCHK(hipStreamSynchronize(st));
  DevState ds;
  DevInfo di;
  HIPCHK(hipMemcpy(&ds, s->w.st, sizeof(ds), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(&di, s->w.info, sizeof(di), hipMemcpyDeviceToHost));
  if (ds.status != 0) {
    // report a device error and clear it: the state keeps its committed pair
    if (clear_status(s->w.st, ds, st) != hipSuccess) return EIG_EDEVICE;
    return status_from_bits(ds.status);
  }
  if (di.n_s != di.n_d) return EIG_EUNSUPPORTED;
  if (n_xi > di.n_d) return EIG_EINVAL;
  const int n_d = di.n_d, N = n_d - (int)n_xi;
  // the members live in W when it is large enough, else in a temporary buffer
  const size_t need = chain_ws_doubles(n_d);
  double* ws = w.W;
  double* tmp = nullptr;
  if (need > n * n) {
    if (hipMalloc(&tmp, need * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      return EIG_ENOMEM;
    }
    ws = tmp;
  }
  struct Free {
    double* p;
    ~Free() {
      if (p) (void)hipFree(p);
    }
  } free_tmp{tmp};
  HIPCHK(launch_chain(w, n_d, xi, (int)n_xi, ws, &w.info->alpha_bad, st));
  HIPCHK(hipStreamSynchronize(st));
  int out[2];
  int bad = 0;
  HIPCHK(hipMemcpy(out, ws + 3 * (size_t)n_d + 1, sizeof(out), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(&bad, &w.info->alpha_bad, sizeof(int), hipMemcpyDeviceToHost));
  if (bad) return EIG_EINVAL;
  const int levels = out[0];
  HIPCHK(launch_chain_count(w, n_d, xi, (int)n_xi, ws, levels, x, (int)n_x, counts, st));
  if (c_max > 0)
    HIPCHK(hipMemcpyAsync(c_out, ws + 2 * (size_t)n_d,
                          (size_t)std::min<int64_t>(c_max, levels) * sizeof(double),
                          hipMemcpyDeviceToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  info->n_poles = N;
  info->levels = levels;
  info->complete = out[1];
  info->lower_bound = out[1] ? N : (int64_t)levels - 2;
  info->n_deflated = (int64_t)n - n_d;
  info->reserved = 0;
  s->last_k = (int)k;
  s->last_p = __builtin_popcount((unsigned)mask);
  s->last_q = (int)k - s->last_p;
  return EIG_OK;
}

int eig_perturb_first_order(eig_state_t s, int64_t k, const double* K, int64_t ldk,
                            const int8_t* sigma, uint32_t mode, double* lambda_out,
                            double* V_out, int64_t ldv, void* hip_stream) {
  TraceRange trace("eig_perturb_first_order");
  if (!s || !K || !sigma || !lambda_out || !V_out || k < 1 || ldk < s->n || ldv < s->n ||
      s->lean)
    return EIG_EINVAL;
  if (k > EIG_KMAX) return EIG_EUNSUPPORTED;
  if (k > s->n) return EIG_EINVAL;
  if (mode & ~(uint32_t)EIG_HOST_INPUT) return EIG_EUNSUPPORTED;
  int mask = 0;
  for (int64_t c = 0; c < k; ++c) {
    if (sigma[c] == 1)
      mask |= 1 << c;
    else if (sigma[c] != -1)
      return EIG_EINVAL;
  }
  if (!s->uploaded) return EIG_ESTATE;
  DeviceGuard g(s->device);
  if (!g.ok) return EIG_EDEVICE;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const size_t n = (size_t)s->n;
  const double* Kd = K;
  int64_t ldkd = ldk;
  if (mode & EIG_HOST_INPUT) {
    HIPCHK(hipMemcpy2DAsync(s->Kbuf, n * sizeof(double), K, (size_t)ldk * sizeof(double),
                            n * sizeof(double), (size_t)k, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    Kd = s->Kbuf;
    ldkd = (int64_t)n;
  }
  Work w = make_work(s, (int)k, Kd, (int)ldkd, mask, true);
  HIPCHK(launch_qtk(w, st));
  HIPCHK(launch_perturb_w(w, lambda_out, st));
  HIPCHK(launch_dgemm((int)n, (int)n, (int)n, w.Q_in, (int)n, w.W, (int)n, V_out, (int)ldv,
                      &w.st->status, st));
  return EIG_OK;
}

int eig_query(eig_state_t s, double* lambda_out, double* Q_out, int64_t ldq,
              int32_t ptrs_on_device, eig_info* info, void* hip_stream) {
  TraceRange trace("eig_query");
  if (!s) return EIG_EINVAL;
  if (Q_out && ldq < s->n) return EIG_EINVAL;
  DeviceGuard g(s->device);
  if (!g.ok) return EIG_EDEVICE;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  HIPCHK(hipStreamSynchronize(st));
  DevState ds;
  DevInfo di;
  HIPCHK(hipMemcpy(&ds, s->w.st, sizeof(ds), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(&di, s->w.info, sizeof(di), hipMemcpyDeviceToHost));
  int rc = EIG_OK;
  if (ds.status != 0) {
    rc = status_from_bits(ds.status);
    HIPCHK(clear_status(s->w.st, ds, st));
    s->enq_gen = ds.gen;
    s->last_vo = false;
  }
  const size_t n = (size_t)s->n;
  const int cur = (int)(ds.gen & 1);
  const hipMemcpyKind kind = ptrs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (lambda_out && s->uploaded) {
    const double* src = s->last_vo ? s->lam_vo : s->lam[cur];
    HIPCHK(hipMemcpyAsync(lambda_out, src, n * sizeof(double), kind, st));
  }
  if (Q_out && s->uploaded) {
    HIPCHK(hipMemcpy2DAsync(Q_out, (size_t)ldq * sizeof(double), s->Q[cur], n * sizeof(double),
                            n * sizeof(double), n, kind, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  if (info) {
    memset(info, 0, sizeof(*info));
    info->n = s->n;
    info->k = s->last_k;
    if (s->last_k > 0) {
      info->p = s->last_p;
      info->q = s->last_q;
      info->n_deflated_rows = di.n_defl;
      info->n_deflated_groups = di.n_groups;
      info->n_segments = di.n_s;
      info->iters_min = (di.n_d > 0) ? di.it_min : 0;
      info->iters_max = di.it_max;
      info->iters_mean = (di.n_d > 0) ? (double)di.it_sum / (double)di.n_d : 0.0;
      info->defl_backward_err = di.bwd;
      info->anorm_bound = di.ahat;
      info->located_by_residues = di.loc_alpha;
    }
    info->generation = ds.gen;
    if (s->timed) {
      for (int i = 0; i < 7; ++i) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, s->ev[i], s->ev[i + 1]) == hipSuccess) info->ms[i] = ms;
      }
      float tot = 0.0f;
      if (hipEventElapsedTime(&tot, s->ev[0], s->ev[8]) == hipSuccess) info->ms[7] = tot;
    }
  }
  return rc;
}

int eig_debug_fetch(eig_state_t s, int32_t what, void* dst, int64_t bytes, void* hip_stream) {
  if (!s || !dst || bytes < 0) return EIG_EINVAL;
  DeviceGuard g(s->device);
  if (!g.ok) return EIG_EDEVICE;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  HIPCHK(hipStreamSynchronize(st));
  DevInfo di;
  HIPCHK(hipMemcpy(&di, s->w.info, sizeof(di), hipMemcpyDeviceToHost));
  const size_t n = (size_t)s->n;
  const Work& w = s->w;
  const void* src = nullptr;
  size_t need = 0;
  switch (what) {
    case EIG_DBG_U:
      if (s->last_k > EIG_KMAX) return EIG_EINVAL;  // a chained update keeps only its last part
      src = w.U;
      need = n * (size_t)s->last_k * sizeof(double);
      break;
    case EIG_DBG_POLE_COUNT: src = w.nu; need = (size_t)di.n_s * sizeof(int); break;
    case EIG_DBG_SEG_START: src = w.seg_start; need = (size_t)(di.n_s + 1) * sizeof(int); break;
    case EIG_DBG_REDUCED_D: src = w.rd; need = (size_t)di.n_d * sizeof(double); break;
    case EIG_DBG_REDUCED_ROW: src = w.rrow; need = (size_t)di.n_d * sizeof(int); break;
    case EIG_DBG_ROOT_ORIGIN: src = w.root_o; need = (size_t)di.n_d * sizeof(int); break;
    case EIG_DBG_ROOT_TAU: src = w.root_tau; need = (size_t)di.n_d * sizeof(double); break;
    case EIG_DBG_ROOT_ITERS: src = w.root_it; need = (size_t)di.n_d * sizeof(int); break;
    case EIG_DBG_W: src = w.W; need = n * n * sizeof(double); break;
    default: return EIG_EINVAL;
  }
  if ((size_t)bytes < need) return EIG_EINVAL;
  if (need > 0) HIPCHK(hipMemcpy(dst, src, need, hipMemcpyDeviceToHost));
  return EIG_OK;
}

}  // extern "C"
