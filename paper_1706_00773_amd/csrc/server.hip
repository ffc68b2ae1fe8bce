// server.hip -- a serving loop for many resident decompositions (C ABI in
// include/eigupd.h): requests (matrix, k, K, sigma) arrive on the host at any
// time; a scheduler thread admits them by device-memory footprint, forms
// batches continuously and runs them as batched updates on several streams,
// so that batches formed while others are on the GPU overlap with them.
//
// Memory.  Each resident decomposition owns a lean state (lambda, O(n k)
// workspace) and one n x n buffer of the device arena holding its current Q.
// An admitted update borrows two more arena buffers, W and Q' (16 n^2 bytes,
// its transient footprint).  When the update has committed, the old Q buffer
// and W go back to the arena and Q' is the matrix's Q; if the update failed
// on the device, Q' and W go back and Q is unchanged.  A request is admitted
// only when its transient buffers fit in the arena; the first-fit arena
// coalesces freed neighbours.  As buffers change roles the free space can split
// into holes; when a request waits with nothing in flight, the resident Q
// buffers are slid to the bottom of the arena (compaction) and it is retried.
//
// Order.  Requests of one matrix are applied in arrival order, one at a time
// (an update reads the Q its predecessor committed).  Requests of different
// matrices are independent and are batched together, up to max_batch per
// batch, oldest first.
//
// Products.  Batches run with EIG_QW_FARFIELD: matrices with n >= 2048 form
// Q' = Q W by the far-field product (its buffers, outside the arena, are
// allocated on the matrix's first update and kept), the others by the grouped
// dense product.
//
// Streams.  Each of the server's streams has its own batch context (fixed
// knobs: persistent root solver, no graphs -- the batch shapes of a request
// stream rarely repeat), pinned staging for the batch's K matrices and a
// completion record; a new batch starts on any stream whose previous batch has
// retired.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "eigupd.h"
#include "internal.h"
#include "state.h"
#include "trace.h"

using namespace eigupd;

namespace {

constexpr size_t ALIGN = 256;

size_t align_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

// First-fit allocator over one device allocation; free blocks kept by offset
// and merged with free neighbours.
class Arena {
 public:
  size_t size = 0;
  size_t used = 0, peak = 0;
  char* base = nullptr;

  void init(char* b, size_t n) {
    base = b;
    size = n;
    free_.clear();
    free_[0] = n;
  }
  // returns SIZE_MAX if no free block is large enough
  size_t alloc(size_t bytes) {
    bytes = align_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first, rem = it->second - bytes;
        free_.erase(it);
        if (rem) free_[off + bytes] = rem;
        used += bytes;
        peak = std::max(peak, used);
        return off;
      }
    }
    return SIZE_MAX;
  }
  void release(size_t off, size_t bytes) {
    bytes = align_up(bytes);
    used -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  double* ptr(size_t off) const { return reinterpret_cast<double*>(base + off); }
  // after a compaction: [0, top) used, the rest one free block
  void reset_free(size_t top) {
    free_.clear();
    if (top < size) free_[top] = size - top;
  }

 private:
  std::map<size_t, size_t> free_;
};

// Moves `bytes` from src down to dst < src inside one allocation: forward
// copies of at most src - dst bytes never overwrite source bytes not yet read.
// The copies are enqueued in order on `st` (the caller synchronises it).
bool move_down(char* dst, const char* src, size_t bytes, hipStream_t st) {
  const size_t gap = (size_t)(src - dst);
  for (size_t pos = 0; pos < bytes; pos += gap) {
    const size_t c = std::min(gap, bytes - pos);
    if (hipMemcpyAsync(dst + pos, src + pos, c, hipMemcpyDeviceToDevice, st) != hipSuccess)
      return false;
  }
  return true;
}

struct Request {
  int64_t id = 0;
  int matrix = 0;
  int k = 0;
  int8_t sigma[EIG_KMAX] = {};
  std::vector<double> K;  // n x k column-major host copy
  double t_submit = 0.0, t_admit = 0.0;
  size_t w_off = 0, q_off = 0;
};

struct Matrix {
  eig_state_s* st = nullptr;
  int n = 0;
  size_t q_off = 0;  // arena offset of the current Q
  bool busy = false;
  bool broken = false;  // an update failed; later ones are refused until a read
};

struct Slot {                  // one stream
  hipStream_t stream = nullptr;
  eig_batch_t batch = nullptr;
  hipEvent_t done = nullptr;
  double* h_K = nullptr;       // pinned staging of the batch's K matrices
  double* d_K = nullptr;       // device copy
  size_t k_cap = 0;            // doubles
  DevState* h_st = nullptr;    // pinned completion records
  std::vector<Request*> running;
};

}  // namespace

struct eig_server_s {
  int device = 0;
  int max_batch = 0;
  void* d_arena = nullptr;
  Arena arena;
  std::vector<Matrix> mats;
  int n_max = 0;
  size_t resident_q = 0;
  std::vector<Slot> slots;
  std::list<Request*> pending;  // arrival order
  std::deque<eig_completion> done;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread worker;
  bool stop = false;
  int in_flight = 0;
  int64_t submitted = 0, completed = 0, failed = 0, batches = 0, batched_updates = 0;
  int64_t compactions = 0;
  std::chrono::steady_clock::time_point t0;
  int worker_error = 0;
};

namespace {

double now_s(const eig_server_s* s) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

int status_of(int bits) { return status_code(bits); }

// Called with the lock held: finish the batch of slot i (its event has fired).
void retire(eig_server_s* s, Slot& sl) {
  const double t = now_s(s);
  for (size_t i = 0; i < sl.running.size(); ++i) {
    Request* r = sl.running[i];
    Matrix& m = s->mats[r->matrix];
    eig_state_s* st = m.st;
    const DevState ds = sl.h_st[i];
    const size_t nn = (size_t)m.n * m.n * sizeof(double);
    int rc = status_of(ds.status);
    if (rc == EIG_OK && ds.gen == st->enq_gen) {
      s->arena.release(m.q_off, nn);  // the old Q
      m.q_off = r->q_off;
    } else {
      if (rc == EIG_OK) rc = EIG_EDEVICE;
      m.broken = true;
      s->arena.release(r->q_off, nn);
      // clear the sticky bits so that the matrix takes later updates; the copy
      // must have landed before any stream runs the matrix's next update
      DevState z = ds;
      z.status = 0;
      if (hipMemcpyAsync(st->w.st, &z, sizeof(z), hipMemcpyHostToDevice, sl.stream) !=
              hipSuccess ||
          hipStreamSynchronize(sl.stream) != hipSuccess)
        rc = EIG_EDEVICE;
      st->enq_gen = ds.gen;
    }
    s->arena.release(r->w_off, nn);
    const int cur = (int)(st->enq_gen & 1);
    st->Q[cur] = s->arena.ptr(m.q_off);
    st->Q[cur ^ 1] = nullptr;
    st->w.W = nullptr;
    m.busy = false;
    eig_completion c;
    memset(&c, 0, sizeof c);
    c.request_id = r->id;
    c.matrix = r->matrix;
    c.status = rc;
    c.t_submit = r->t_submit;
    c.t_admit = r->t_admit;
    c.t_done = t;
    c.batch_size = (int32_t)sl.running.size();
    s->done.push_back(c);
    s->completed += 1;
    if (rc != EIG_OK) s->failed += 1;
    delete r;
  }
  s->in_flight -= (int)sl.running.size();
  sl.running.clear();
  s->cv_done.notify_all();
}

// Called with the lock held and nothing in flight: slides every resident Q to
// the bottom of the arena (in offset order) so that the free space is one
// block.  The moves run on the first slot's stream, which is synchronised
// before returning: the server's streams do not wait for one another (nor for
// the null stream, on which a device-to-device hipMemcpy may still be running
// when it returns), and the next batch reads the moved buffers.  Returns false
// if a device copy failed.
bool compact(eig_server_s* s) {
  hipStream_t st = s->slots[0].stream;
  std::vector<int> order(s->mats.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::sort(order.begin(), order.end(),
            [&](int a, int b) { return s->mats[a].q_off < s->mats[b].q_off; });
  size_t top = 0;
  for (int i : order) {
    Matrix& m = s->mats[i];
    const size_t bytes = align_up((size_t)m.n * m.n * sizeof(double));
    if (m.q_off != top) {
      if (!move_down(s->arena.base + top, s->arena.base + m.q_off, bytes, st)) return false;
      m.q_off = top;
      m.st->Q[m.st->enq_gen & 1] = s->arena.ptr(top);
    }
    top += bytes;
  }
  if (hipStreamSynchronize(st) != hipSuccess) return false;
  s->arena.reset_free(top);
  s->compactions += 1;
  return true;
}

void fail_request(eig_server_s* s, Request* r, int rc) {
  eig_completion c;
  memset(&c, 0, sizeof c);
  c.request_id = r->id;
  c.matrix = r->matrix;
  c.status = rc;
  c.t_submit = r->t_submit;
  c.t_admit = c.t_done = now_s(s);
  s->done.push_back(c);
  s->completed += 1;
  s->failed += 1;
  delete r;
  s->cv_done.notify_all();
}

// Called with the lock held: admit what fits and launch it on slot `sl`.  A
// request of a matrix whose earlier update failed completes at once with
// EIG_EDEPENDENCY.  Returns the number of requests launched or completed so
// (or -1 on a launch failure).
int launch(eig_server_s* s, Slot& sl) {
  TraceRange trace("eig_server.launch");
  std::vector<Request*> pick;
  std::vector<char> blocked(s->mats.size(), 0);  // head request waits for memory
  size_t kdoubles = 0;
  bool first = true;
  int ndep = 0;
  for (auto it = s->pending.begin(); it != s->pending.end() && (int)pick.size() < s->max_batch;) {
    Request* r = *it;
    Matrix& m = s->mats[r->matrix];
    if (!m.busy && m.broken) {
      // its predecessor failed: not applied (the matrix keeps its state)
      it = s->pending.erase(it);
      fail_request(s, r, EIG_EDEPENDENCY);
      ++ndep;
      continue;
    }
    const bool oldest = first;
    first = false;
    if (m.busy || blocked[r->matrix]) {
      ++it;
      continue;
    }
    const size_t nn = (size_t)m.n * m.n * sizeof(double);
    const size_t kd = (size_t)m.n * r->k;
    if (kdoubles + kd > sl.k_cap) break;
    size_t w_off = s->arena.alloc(nn), q_off = SIZE_MAX;
    if (w_off != SIZE_MAX) {
      q_off = s->arena.alloc(nn);
      if (q_off == SIZE_MAX) s->arena.release(w_off, nn);
    }
    if (q_off == SIZE_MAX) {
      // no room: the oldest request keeps its turn (nothing younger is
      // admitted ahead of it); any other one waits behind its matrix
      if (oldest) break;
      blocked[r->matrix] = 1;
      ++it;
      continue;
    }
    r->w_off = w_off;
    r->q_off = q_off;
    m.busy = true;
    kdoubles += kd;
    pick.push_back(r);
    it = s->pending.erase(it);
  }
  if (pick.empty()) return ndep;
  // stage the K matrices, build the items
  std::vector<eig_batch_item> items(pick.size());
  size_t o = 0;
  const double t = now_s(s);
  for (size_t i = 0; i < pick.size(); ++i) {
    Request* r = pick[i];
    Matrix& m = s->mats[r->matrix];
    eig_state_s* st = m.st;
    memcpy(sl.h_K + o, r->K.data(), r->K.size() * sizeof(double));
    items[i].state = st;
    items[i].k = r->k;
    items[i].K = sl.d_K + o;
    items[i].ldk = m.n;
    memcpy(items[i].sigma, r->sigma, sizeof r->sigma);
    o += r->K.size();
    const int cur = (int)(st->enq_gen & 1);
    st->Q[cur] = s->arena.ptr(m.q_off);
    st->Q[cur ^ 1] = s->arena.ptr(r->q_off);
    st->w.W = s->arena.ptr(r->w_off);
    r->t_admit = t;
  }
  hipError_t e = hipMemcpyAsync(sl.d_K, sl.h_K, o * sizeof(double), hipMemcpyHostToDevice,
                                sl.stream);
  int rc = (e == hipSuccess)
               ? eig_update_batch(sl.batch, items.data(), (int32_t)items.size(), EIG_QW_FARFIELD,
                                  sl.stream)
               : EIG_EDEVICE;
  if (rc == EIG_OK) {
    for (size_t i = 0; i < pick.size(); ++i) {
      e = hipMemcpyAsync(&sl.h_st[i], s->mats[pick[i]->matrix].st->w.st, sizeof(DevState),
                         hipMemcpyDeviceToHost, sl.stream);
      if (e != hipSuccess) rc = EIG_EDEVICE;
    }
    if (hipEventRecord(sl.done, sl.stream) != hipSuccess) rc = EIG_EDEVICE;
  }
  if (rc != EIG_OK) {
    // nothing of this batch will complete: give the buffers back, fail the requests
    for (Request* r : pick) {
      Matrix& m = s->mats[r->matrix];
      const size_t nn = (size_t)m.n * m.n * sizeof(double);
      s->arena.release(r->w_off, nn);
      s->arena.release(r->q_off, nn);
      m.busy = false;
      fail_request(s, r, rc);
    }
    s->worker_error = rc;
    return -1;
  }
  sl.running = pick;
  s->in_flight += (int)pick.size();
  s->batches += 1;
  s->batched_updates += (int64_t)pick.size();
  return (int)pick.size() + ndep;
}

void worker_main(eig_server_s* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    bool progressed = false;
    for (Slot& sl : s->slots) {
      if (!sl.running.empty() && hipEventQuery(sl.done) == hipSuccess) {
        retire(s, sl);
        progressed = true;
      }
    }
    if (s->worker_error == 0) {
      for (Slot& sl : s->slots) {
        if (!sl.running.empty() || s->pending.empty()) continue;
        const int got = launch(s, sl);
        if (got > 0) progressed = true;
        if (got < 0) break;
      }
    }
    // nothing running and nothing admitted: the free space may be split into
    // holes; compact the arena and try again before failing the oldest request
    if (s->in_flight == 0 && !s->pending.empty() && !progressed && s->worker_error == 0) {
      if (!compact(s)) {
        s->worker_error = EIG_EDEVICE;
      } else if (launch(s, s->slots[0]) > 0) {
        progressed = true;
      } else if (s->in_flight == 0) {
        fail_request(s, s->pending.front(), EIG_ENOMEM);
        s->pending.pop_front();
        progressed = true;
      }
    }
    if (s->worker_error) {
      while (!s->pending.empty()) {
        fail_request(s, s->pending.front(), s->worker_error);
        s->pending.pop_front();
      }
    }
    if (s->stop && s->pending.empty() && s->in_flight == 0) break;
    if (progressed) continue;
    if (s->in_flight > 0) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    } else {
      s->cv_work.wait(lk, [&] { return s->stop || !s->pending.empty(); });
    }
  }
}

}  // namespace

extern "C" {

int eig_server_create(eig_server_t* out, int32_t device, int64_t arena_bytes, int32_t max_batch,
                      int32_t streams, int64_t max_k_doubles) {
  if (!out || arena_bytes < (int64_t)ALIGN || max_batch < 1 || max_batch > 4096 || streams < 1 ||
      streams > 8 || max_k_doubles < 1)
    return EIG_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return EIG_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return EIG_EDEVICE;
  eig_server_s* s = new (std::nothrow) eig_server_s();
  if (!s) return EIG_ENOMEM;
  s->device = device;
  s->max_batch = max_batch;
  s->t0 = std::chrono::steady_clock::now();
  bool ok = hipMalloc(&s->d_arena, (size_t)arena_bytes) == hipSuccess;
  if (ok) s->arena.init(static_cast<char*>(s->d_arena), (size_t)arena_bytes);
  s->slots.resize(streams);
  for (Slot& sl : s->slots) {
    if (!ok) break;
    sl.k_cap = (size_t)max_k_doubles;
    ok = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess &&
         hipHostMalloc(reinterpret_cast<void**>(&sl.h_K), sl.k_cap * sizeof(double),
                       hipHostMallocDefault) == hipSuccess &&
         hipMalloc(reinterpret_cast<void**>(&sl.d_K), sl.k_cap * sizeof(double)) == hipSuccess &&
         hipHostMalloc(reinterpret_cast<void**>(&sl.h_st), (size_t)max_batch * sizeof(DevState),
                       hipHostMallocDefault) == hipSuccess &&
         eig_batch_create(&sl.batch, max_batch, device) == EIG_OK;
    if (ok) {
      eig_batch_set(sl.batch, EIG_KNOB_ROOTSOLVE, EIG_ROOTSOLVE_PERSISTENT);
      eig_batch_set(sl.batch, EIG_KNOB_GEMM_TILE, 128);
      eig_batch_set(sl.batch, EIG_KNOB_GRAPHS, 0);
    }
  }
  if (!ok) {
    (void)hipGetLastError();
    eig_server_destroy(s);
    return EIG_ENOMEM;
  }
  s->worker = std::thread(worker_main, s);
  *out = s;
  return EIG_OK;
}

int eig_server_destroy(eig_server_t s) {
  if (!s) return EIG_EINVAL;
  if (s->worker.joinable()) {
    {
      std::lock_guard<std::mutex> g(s->mu);
      s->stop = true;
    }
    s->cv_work.notify_all();
    s->worker.join();
  }
  (void)hipSetDevice(s->device);
  (void)hipDeviceSynchronize();
  for (Request* r : s->pending) delete r;
  for (Matrix& m : s->mats)
    if (m.st) {
      m.st->Q[0] = m.st->Q[1] = nullptr;
      m.st->w.W = nullptr;
      eig_state_destroy(m.st);
    }
  for (Slot& sl : s->slots) {
    if (sl.batch) eig_batch_destroy(sl.batch);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.h_K) (void)hipHostFree(sl.h_K);
    if (sl.h_st) (void)hipHostFree(sl.h_st);
    if (sl.d_K) (void)hipFree(sl.d_K);
  }
  if (s->d_arena) (void)hipFree(s->d_arena);
  delete s;
  return EIG_OK;
}

int eig_server_add(eig_server_t s, int64_t n, const double* lambda, const double* Q, int64_t ldq,
                   int32_t ptrs_on_device, int32_t* matrix) {
  if (!s || !lambda || !Q || !matrix || n < 1 || n > 65536 || ldq < n) return EIG_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  (void)hipSetDevice(s->device);
  const size_t nn = (size_t)n * n * sizeof(double);
  // the arena must keep room for one update of the largest matrix
  const int nmax = std::max(s->n_max, (int)n);
  const size_t need = align_up(nn) + s->resident_q + 2 * align_up((size_t)nmax * nmax * 8);
  if (need > s->arena.size) return EIG_ENOMEM;
  const size_t q_off = s->arena.alloc(nn);
  if (q_off == SIZE_MAX) return EIG_ENOMEM;
  eig_state_t st = nullptr;
  int rc = state_create(&st, n, s->device, true);
  if (rc != EIG_OK) {
    s->arena.release(q_off, nn);
    return rc;
  }
  // lambda (checked ascending and finite, as on upload) and Q into place
  std::vector<double> h((size_t)n);
  const hipMemcpyKind kind = ptrs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  bool ok = hipMemcpy(h.data(), lambda, (size_t)n * sizeof(double),
                      ptrs_on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost) == hipSuccess;
  for (int64_t j = 0; ok && j < n; ++j)
    if (!std::isfinite(h[j]) || (j > 0 && !(h[j] >= h[j - 1]))) rc = EIG_ENOTSORTED;
  if (ok && rc == EIG_OK) {
    ok = hipMemcpy(st->lam[0], h.data(), (size_t)n * sizeof(double), hipMemcpyHostToDevice) ==
             hipSuccess &&
         hipMemcpy2D(s->arena.ptr(q_off), (size_t)n * sizeof(double), Q,
                     (size_t)ldq * sizeof(double), (size_t)n * sizeof(double), (size_t)n,
                     kind) == hipSuccess;
    DevState z{};
    ok = ok && hipMemcpy(st->w.st, &z, sizeof(z), hipMemcpyHostToDevice) == hipSuccess;
    // the copies above may still be in flight (device-to-device, or the DMA of
    // a staged host copy); the server's streams do not wait for them
    ok = ok && hipDeviceSynchronize() == hipSuccess;
  }
  if (!ok || rc != EIG_OK) {
    s->arena.release(q_off, nn);
    eig_state_destroy(st);
    return ok ? rc : EIG_EDEVICE;
  }
  st->Q[0] = s->arena.ptr(q_off);
  st->enq_gen = 0;
  st->uploaded = true;
  Matrix m;
  m.st = st;
  m.n = (int)n;
  m.q_off = q_off;
  s->mats.push_back(m);
  s->n_max = nmax;
  s->resident_q += align_up(nn);
  *matrix = (int32_t)s->mats.size() - 1;
  return EIG_OK;
}

int eig_server_submit(eig_server_t s, int32_t matrix, int64_t k, const double* K, int64_t ldk,
                      const int8_t* sigma, int64_t request_id) {
  if (!s || !K || !sigma || k < 1) return EIG_EINVAL;
  if (k > EIG_KMAX) return EIG_EUNSUPPORTED;
  Request* r = new (std::nothrow) Request();
  if (!r) return EIG_ENOMEM;
  int n = 0;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (matrix < 0 || matrix >= (int)s->mats.size()) {
      delete r;
      return EIG_EINVAL;
    }
    n = s->mats[matrix].n;
  }
  if (ldk < n || k > n || (size_t)n * k > s->slots[0].k_cap) {
    delete r;
    return EIG_EINVAL;
  }
  for (int c = 0; c < k; ++c) {
    if (sigma[c] != 1 && sigma[c] != -1) {
      delete r;
      return EIG_EINVAL;
    }
    r->sigma[c] = sigma[c];
  }
  r->id = request_id;
  r->matrix = matrix;
  r->k = (int)k;
  r->K.resize((size_t)n * k);
  for (int64_t c = 0; c < k; ++c)
    memcpy(r->K.data() + (size_t)c * n, K + (size_t)c * ldk, (size_t)n * sizeof(double));
  {
    std::lock_guard<std::mutex> g(s->mu);
    r->t_submit = now_s(s);
    s->pending.push_back(r);
    s->submitted += 1;
  }
  s->cv_work.notify_one();
  return EIG_OK;
}

int eig_server_poll(eig_server_t s, eig_completion* out, int32_t max, int32_t timeout_ms,
                    int32_t* count) {
  if (!s || !count || max < 0 || (max > 0 && !out)) return EIG_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && timeout_ms > 0)
    s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [&] { return !s->done.empty(); });
  int c = 0;
  while (c < max && !s->done.empty()) {
    out[c++] = s->done.front();
    s->done.pop_front();
  }
  *count = c;
  return EIG_OK;
}

int eig_server_drain(eig_server_t s) {
  if (!s) return EIG_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->pending.empty() && s->in_flight == 0; });
  return s->worker_error;
}

int eig_server_read(eig_server_t s, int32_t matrix, double* lambda_out, double* Q_out,
                    int64_t ldq, int32_t ptrs_on_device) {
  if (!s) return EIG_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  if (matrix < 0 || matrix >= (int)s->mats.size()) return EIG_EINVAL;
  Matrix& m = s->mats[matrix];
  if (Q_out && ldq < m.n) return EIG_EINVAL;
  // wait until no update of this matrix is queued or running
  s->cv_done.wait(lk, [&] {
    if (m.busy) return false;
    for (Request* r : s->pending)
      if (r->matrix == matrix) return false;
    return true;
  });
  (void)hipSetDevice(s->device);
  m.broken = false;  // the caller has seen the state a failed update left
  const int cur = (int)(m.st->enq_gen & 1);
  const hipMemcpyKind kind = ptrs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (lambda_out &&
      hipMemcpy(lambda_out, m.st->lam[cur], (size_t)m.n * sizeof(double), kind) != hipSuccess)
    return EIG_EDEVICE;
  if (Q_out && hipMemcpy2D(Q_out, (size_t)ldq * sizeof(double), s->arena.ptr(m.q_off),
                           (size_t)m.n * sizeof(double), (size_t)m.n * sizeof(double),
                           (size_t)m.n, kind) != hipSuccess)
    return EIG_EDEVICE;
  // device-to-device copies may return before they finish
  if (ptrs_on_device && hipDeviceSynchronize() != hipSuccess) return EIG_EDEVICE;
  return EIG_OK;
}

int eig_server_stats(eig_server_t s, eig_server_info* info) {
  if (!s || !info) return EIG_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  memset(info, 0, sizeof *info);
  info->matrices = (int64_t)s->mats.size();
  info->submitted = s->submitted;
  info->completed = s->completed;
  info->failed = s->failed;
  info->queued = (int64_t)s->pending.size();
  info->in_flight = s->in_flight;
  info->batches = s->batches;
  info->mean_batch = s->batches ? (double)s->batched_updates / (double)s->batches : 0.0;
  info->arena_bytes = (int64_t)s->arena.size;
  info->resident_bytes = (int64_t)s->resident_q;
  info->arena_used = (int64_t)s->arena.used;
  info->arena_peak = (int64_t)s->arena.peak;
  info->compactions = s->compactions;
  return EIG_OK;
}

}  // extern "C"
