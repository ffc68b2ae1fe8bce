// noalloc.hip -- eig_eigvals_rankk_noalloc: the eigenvalues of
// A + K Sigma K^T (Sec. 2.1-2.3) from a decomposition the caller holds, with
// every intermediate in one static device array instead of allocated memory.
//
// The kernels are those of eig_update_rankk with EIG_VALUES_ONLY (U = Q^T K,
// deflation, pole counts and location, root refinement, the ordered merge);
// only the place of their workspace differs.  The array `scratch` below holds
// that workspace for one update of order n <= EIG_NOALLOC_NMAX.  In host code
// the name `scratch` is not a device address: its address on each device is
// taken once, with that device current, by hipGetSymbolAddress, and only that
// address is handed to kernels.
#include <mutex>

#include "common.h"
#include "state.h"

// U, deflation, reduced problem, roots, column parameters, status and info of
// one update of order up to EIG_NOALLOC_NMAX (about 600 bytes per row at rank
// up to 8).  Each device keeps its own copy until the process ends; calls on
// one device share it.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(10) << 20;
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

using namespace eigupd;

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};  // address of scratch on each device

// The device address of scratch on the current device `dev`, looked up once.
int scratch_address(int dev, char** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return EIG_EDEVICE;
    }
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return EIG_OK;
}

// The sticky error bits of the update as an EIG_* code in the caller's word.
__global__ void noalloc_status_kernel(const DevState* st, int32_t* out) {
  *out = status_code(st->status);
}

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

#define HIPCHK(x)                              \
  do {                                         \
    if ((x) != hipSuccess) return EIG_EDEVICE; \
  } while (0)

}  // namespace

extern "C" int eig_eigvals_rankk_noalloc(int64_t n, int64_t k, const double* lambda,
                                         const double* Q, int64_t ldq, const double* K,
                                         int64_t ldk, const int8_t* sigma, uint32_t mode,
                                         double* lambda_out, int32_t* status_out,
                                         int32_t device, void* hip_stream) {
  if (!lambda || !Q || !K || !sigma || !lambda_out || !status_out || n < 1 || k < 1 ||
      ldq < n || ldk < n)
    return EIG_EINVAL;
  if (n > EIG_NOALLOC_NMAX || k > EIG_KMAX) return EIG_EUNSUPPORTED;
  if (k > n || ldq > INT32_MAX || ldk > INT32_MAX) return EIG_EINVAL;
  if (mode & ~(uint32_t)EIG_LOCATE_RESIDUES) return EIG_EUNSUPPORTED;
  int mask = 0;
  for (int64_t c = 0; c < k; ++c) {
    if (sigma[c] == 1)
      mask |= 1 << c;
    else if (sigma[c] != -1)
      return EIG_EINVAL;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev ||
      device >= NOALLOC_MAX_DEVICES)
    return EIG_EDEVICE;
  DeviceGuard g(device);
  if (!g.ok) return EIG_EDEVICE;
  char* base = nullptr;
  const int rc = scratch_address(device, &base);
  if (rc != EIG_OK) return rc;
  Work w{};
  if (carve_workspace(w, (size_t)n, nullptr, 0) > NOALLOC_SCRATCH_BYTES) return EIG_EUNSUPPORTED;
  carve_workspace(w, (size_t)n, base, 0);
  w.n = (int)n;
  w.k = (int)k;
  w.ldk = (int)ldk;
  w.ldq = (int)ldq;
  w.max_evals = MAX_EVALS;
  w.sig_pos_mask = mask;
  w.ncols = (int)n;
  w.lam_in = lambda;
  w.Q_in = Q;
  w.K = K;
  w.lam_out = nullptr;
  w.Q_out = nullptr;
  w.lam_fin = lambda_out;
  w.W = nullptr;
  w.lp_part = nullptr;
  w.lp_resid = nullptr;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  // the array keeps the last call's contents: clear the status and the
  // generation (DevState, 4 ints) with a kernel; DevInfo is set by deflation
  hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, st, reinterpret_cast<int*>(w.st),
                     (int)(sizeof(DevState) / sizeof(int)));
  HIPCHK(hipGetLastError());
  HIPCHK(launch_qtk(w, st));
  HIPCHK(launch_deflate(w, st));
  if ((mode & EIG_LOCATE_RESIDUES) && k == 2) HIPCHK(launch_alpha_locate(w, st));
  HIPCHK(launch_polecount(w, st));
  HIPCHK(launch_locate(w, st));
  HIPCHK(launch_rootsolve(w, st));
  HIPCHK(launch_finalize(w, st));
  hipLaunchKernelGGL(noalloc_status_kernel, dim3(1), dim3(1), 0, st, w.st, status_out);
  HIPCHK(hipGetLastError());
  return EIG_OK;
}
