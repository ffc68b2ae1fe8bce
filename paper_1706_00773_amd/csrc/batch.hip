// batch.hip -- batched rank-k updates of several resident states (different n
// and k) with grouped launches, a persistent root solver, hipGraph replay per
// batch shape and an online autotuner (the C ABI is in include/eigupd.h).
//
// One batch runs every phase of the update once for all its instances:
// instances are ordered by (k ascending, n descending); the kernels of one
// phase are launched once per distinct k (the kernels are specialised by k)
// over a descriptor array (Group: Work descriptors + block prefix sums), and
// Q' = Q W is one grouped launch over all instances.  The per-call data
// (descriptors, prefix sums) is copied to a fixed device area before the
// launches, so a graph captured for one batch shape -- the ordered list of
// (k, n), the mode and the tuning choices -- replays for every later batch of
// that shape whatever the states and K are.
//
// Autotuner.  Two knobs, each bitwise neutral (every choice computes the same
// numbers in the same order): the root solver as one block per (instance,
// root block) or as a persistent grid drawing those items from a queue, and
// the tile of the grouped GEMM (128 or 64).  The first two batches of a shape
// run one candidate combination each with HIP events around the two phases;
// the faster candidate of each knob is kept for the shape.  Graphs are
// captured from the second batch of a shape once its choices are fixed.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "eigupd.h"
#include "internal.h"
#include "state.h"
#include "trace.h"

using namespace eigupd;

namespace {

enum { KIND_QTK = 0, KIND_ROOT = 1, KIND_WB = 2, KIND_REFL = 3, KIND_SOLVE = 4, NKIND = 5 };
constexpr int MAX_GRAPHS = 64;

// Per-call device area, laid out from the shape alone (so the pointers a graph
// captures stay valid for every batch of that shape):
//   Work[count] | GemmDesc[count] | prefix sums: for each k present and each
//   kind, cnt[k] + 1 ints; then the GEMM's count + 1 ints.
struct Plan {
  std::vector<int> order;     // instance order (k asc, n desc)
  int cnt[KMAX + 1] = {};     // instances per k
  int off[KMAX + 1] = {};     // first instance of each k
  int blocks[KMAX + 1][NKIND] = {};
  size_t poff[KMAX + 1][NKIND] = {};  // int offsets of the prefix arrays
  size_t gemm_poff = 0;
  size_t gemm_bytes_off = 0, prefix_bytes_off = 0, bytes = 0;
  int gemm_blocks = 0;
  int count = 0;
  std::vector<char> ff;       // per position: Q' = Q W by the far-field product
  std::vector<Work> host_works;  // per position (the far-field launches take them by value)
  std::vector<eig_state_s*> states;  // per position
  bool any_ff = false;
  std::string key;            // shape: mode, then (k, n) per position
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

void layout(Plan& p) {
  p.gemm_bytes_off = align256((size_t)p.count * sizeof(Work));
  p.prefix_bytes_off = p.gemm_bytes_off + align256((size_t)p.count * sizeof(GemmDesc));
  size_t o = 0;
  for (int k = 1; k <= KMAX; ++k)
    for (int kind = 0; kind < NKIND; ++kind) {
      p.poff[k][kind] = o;
      if (p.cnt[k]) o += (size_t)p.cnt[k] + 1;
    }
  p.gemm_poff = o;
  o += (size_t)p.count + 1;
  p.bytes = p.prefix_bytes_off + o * sizeof(int);
}

}  // namespace

struct eig_batch_s {
  int device = 0;
  int max_items = 0;
  int num_cu = 0;
  void* d_block = nullptr;
  int* d_queue = nullptr;
  size_t desc_bytes = 0;  // capacity of the per-call area (see Plan)
  void* h_slot[2] = {nullptr, nullptr};
  hipEvent_t slot_ev[2] = {};
  int slot = 0;
  hipStream_t cap = nullptr;
  hipEvent_t tev[4] = {};
  // the per-rank chains of a batch with several ranks run on side streams,
  // forked from and joined back into the caller's stream
  hipStream_t side[KMAX + 1] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[KMAX + 1] = {};
  struct Entry {
    int seen = 0;
    hipGraphExec_t exec = nullptr;
  };
  std::map<std::string, Entry> graphs;
  struct Tune {
    int phase = 0;
    float root_ms[2] = {0.0f, 0.0f};
    float gemm_ms[2] = {0.0f, 0.0f};
    int root = 0, tile = 0;
    bool done = false;
  };
  std::map<std::string, Tune> tune;
  int force_root = EIG_AUTO, force_tile = EIG_AUTO, use_graphs = 1;
  int last_root = 0, last_tile = 0, last_graph = 0;
  long long graph_launches = 0;
};

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

// upper bound of Plan::bytes for `max_items` instances
size_t area_bytes(int max_items) {
  return align256((size_t)max_items * sizeof(Work)) +
         align256((size_t)max_items * sizeof(GemmDesc)) +
         ((size_t)NKIND * (max_items + KMAX) + max_items + 1) * sizeof(int);
}

#define HIPCHK(x)                              \
  do {                                         \
    if ((x) != hipSuccess) return EIG_EDEVICE; \
  } while (0)

// Enqueues the whole batch on `st` (direct launches, or recorded into a graph
// when `st` is capturing).  ev: optional events around the root solve and the
// GEMM (4 events, recorded only when non-null).
hipError_t enqueue(eig_batch_s* b, const Plan& p, bool vo, int root_form, int tile,
                   hipStream_t st, const hipEvent_t* ev) {
  hipError_t e = hipSuccess;
  char* base = static_cast<char*>(b->d_block);
  Work* d_works = reinterpret_cast<Work*>(base);
  const GemmDesc* d_gemm = reinterpret_cast<const GemmDesc*>(base + p.gemm_bytes_off);
  const int* d_prefix = reinterpret_cast<const int*>(base + p.prefix_bytes_off);
  auto group = [&](int k, int kind) {
    return Group{d_works + p.off[k], d_prefix + p.poff[k][kind], p.cnt[k]};
  };
#define STEP(x)            \
  do {                     \
    e = (x);               \
    if (e != hipSuccess) return e; \
  } while (0)
  // one rank's phases up to W (the instances of different ranks share nothing
  // until the grouped GEMM)
  const int pgrid = (root_form == EIG_ROOTSOLVE_PERSISTENT) ? 2 * b->num_cu : 0;
  auto chain = [&](int k, hipStream_t cs, bool timed) -> hipError_t {
    hipError_t e2;
#define CSTEP(x)                      \
  do {                                \
    e2 = (x);                         \
    if (e2 != hipSuccess) return e2;  \
  } while (0)
    CSTEP(launch_qtk_group(k, group(k, KIND_QTK), p.blocks[k][KIND_QTK], cs));
    CSTEP(launch_deflate_group(k, d_works + p.off[k], p.cnt[k], cs));
    CSTEP(launch_polecount_group(k, group(k, KIND_ROOT), p.blocks[k][KIND_ROOT], cs));
    CSTEP(launch_locate_group(d_works + p.off[k], p.cnt[k], cs));
    if (timed) CSTEP(hipEventRecord(ev[0], cs));
    CSTEP(launch_rootsolve_group(k, group(k, KIND_SOLVE), p.blocks[k][KIND_SOLVE],
                                 group(k, KIND_ROOT), p.blocks[k][KIND_ROOT], pgrid,
                                 b->d_queue + k, cs));
    if (timed) CSTEP(hipEventRecord(ev[1], cs));
    CSTEP(launch_finalize_group(k, d_works + p.off[k], p.cnt[k], cs));
    if (vo) return hipSuccess;
    CSTEP(launch_wbuild_group(k, group(k, KIND_WB), p.blocks[k][KIND_WB], cs));
    CSTEP(launch_reflect_group(k, group(k, KIND_REFL), p.blocks[k][KIND_REFL], cs));
#undef CSTEP
    return hipSuccess;
  };
  int ranks = 0;
  for (int k = 1; k <= KMAX; ++k) ranks += p.cnt[k] ? 1 : 0;
  if (ev || ranks < 2) {
    // one stream, phase by phase across the ranks (the autotuner's timed runs
    // bracket the root solve of all ranks with its events)
    for (int k = 1; k <= KMAX; ++k)
      if (p.cnt[k]) STEP(launch_qtk_group(k, group(k, KIND_QTK), p.blocks[k][KIND_QTK], st));
    for (int k = 1; k <= KMAX; ++k)
      if (p.cnt[k]) STEP(launch_deflate_group(k, d_works + p.off[k], p.cnt[k], st));
    for (int k = 1; k <= KMAX; ++k)
      if (p.cnt[k])
        STEP(launch_polecount_group(k, group(k, KIND_ROOT), p.blocks[k][KIND_ROOT], st));
    for (int k = 1; k <= KMAX; ++k)
      if (p.cnt[k]) STEP(launch_locate_group(d_works + p.off[k], p.cnt[k], st));
    if (ev) STEP(hipEventRecord(ev[0], st));
    for (int k = 1; k <= KMAX; ++k)
      if (p.cnt[k])
        STEP(launch_rootsolve_group(k, group(k, KIND_SOLVE), p.blocks[k][KIND_SOLVE],
                                    group(k, KIND_ROOT), p.blocks[k][KIND_ROOT], pgrid,
                                    b->d_queue + k, st));
    if (ev) STEP(hipEventRecord(ev[1], st));
    for (int k = 1; k <= KMAX; ++k)
      if (p.cnt[k]) STEP(launch_finalize_group(k, d_works + p.off[k], p.cnt[k], st));
    if (vo) return hipSuccess;
    for (int k = 1; k <= KMAX; ++k)
      if (p.cnt[k])
        STEP(launch_wbuild_group(k, group(k, KIND_WB), p.blocks[k][KIND_WB], st));
    for (int k = 1; k <= KMAX; ++k)
      if (p.cnt[k])
        STEP(launch_reflect_group(k, group(k, KIND_REFL), p.blocks[k][KIND_REFL], st));
  } else {
    // several ranks: the first rank's chain on `st`, the others on side
    // streams forked from it, all joined back before the grouped GEMM (inside
    // a capture the side streams join the graph through the fork event)
    STEP(hipEventRecord(b->fork_ev, st));
    int first = 0;
    for (int k = 1; k <= KMAX; ++k) {
      if (!p.cnt[k]) continue;
      if (!first) {
        first = k;
        continue;
      }
      STEP(hipStreamWaitEvent(b->side[k], b->fork_ev, 0));
      STEP(chain(k, b->side[k], false));
      STEP(hipEventRecord(b->join_ev[k], b->side[k]));
    }
    STEP(chain(first, st, false));
    for (int k = first + 1; k <= KMAX; ++k)
      if (p.cnt[k]) STEP(hipStreamWaitEvent(st, b->join_ev[k], 0));
    if (vo) return hipSuccess;
  }
  if (ev) STEP(hipEventRecord(ev[2], st));
  STEP(launch_dgemm_group(tile, d_gemm, d_prefix + p.gemm_poff, p.count, p.gemm_blocks, st));
  // instances of the far-field product: their own plan, W blocks and products
  // (the grouped launches above gave them no blocks)
  for (int pos = 0; pos < p.count; ++pos) {
    if (!p.ff[pos]) continue;
    const Work& w = p.host_works[pos];
    eig_state_s* s = p.states[pos];
    const FarField f = ff_layout(s->ff_block, w.n, w.k);
    STEP(launch_ff_plan(w, f, st));
    STEP(launch_wbuild_ff(w, f, st));
    STEP(launch_group_reflect(w, st));
    STEP(launch_qw_farfield(w, f, st));
  }
  if (ev) STEP(hipEventRecord(ev[3], st));
  STEP(launch_commit_group(d_works, p.count, st));
#undef STEP
  return hipSuccess;
}

void drop_graphs(eig_batch_s* b) {
  for (auto& kv : b->graphs)
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
  b->graphs.clear();
}

}  // namespace

extern "C" {

int eig_batch_create(eig_batch_t* out, int32_t max_items, int32_t device) {
  if (!out || max_items < 1 || max_items > (1 << 20)) return EIG_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return EIG_EDEVICE;
  DeviceGuard g(device);
  if (!g.ok) return EIG_EDEVICE;
  eig_batch_s* b = new (std::nothrow) eig_batch_s();
  if (!b) return EIG_ENOMEM;
  b->device = device;
  b->max_items = max_items;
  if (hipDeviceGetAttribute(&b->num_cu, hipDeviceAttributeMultiprocessorCount, device) !=
      hipSuccess)
    b->num_cu = 256;
  b->desc_bytes = area_bytes(max_items);
  const size_t qbytes = 256;
  bool ok = hipMalloc(&b->d_block, align256(b->desc_bytes) + qbytes) == hipSuccess;
  for (int i = 0; ok && i < 2; ++i)
    ok = hipHostMalloc(&b->h_slot[i], b->desc_bytes, hipHostMallocDefault) == hipSuccess &&
         hipEventCreateWithFlags(&b->slot_ev[i], hipEventDisableTiming) == hipSuccess;
  for (int i = 0; ok && i < 4; ++i) ok = hipEventCreate(&b->tev[i]) == hipSuccess;
  ok = ok && hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming) == hipSuccess;
  for (int k = 1; ok && k <= KMAX; ++k)
    ok = hipStreamCreateWithFlags(&b->side[k], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&b->join_ev[k], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    eig_batch_destroy(b);
    return EIG_ENOMEM;
  }
  b->d_queue = reinterpret_cast<int*>(static_cast<char*>(b->d_block) + align256(b->desc_bytes));
  for (int i = 0; i < 2; ++i) memset(b->h_slot[i], 0, b->desc_bytes);
  *out = b;
  return EIG_OK;
}

int eig_batch_destroy(eig_batch_t b) {
  if (!b) return EIG_EINVAL;
  {
    DeviceGuard g(b->device);
    (void)hipDeviceSynchronize();
    drop_graphs(b);
    for (auto& e : b->slot_ev)
      if (e) (void)hipEventDestroy(e);
    for (auto& e : b->tev)
      if (e) (void)hipEventDestroy(e);
    for (auto& h : b->h_slot)
      if (h) (void)hipHostFree(h);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (int k = 1; k <= KMAX; ++k) {
      if (b->side[k]) (void)hipStreamDestroy(b->side[k]);
      if (b->join_ev[k]) (void)hipEventDestroy(b->join_ev[k]);
    }
    if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
    if (b->d_block) (void)hipFree(b->d_block);
  }
  delete b;
  return EIG_OK;
}

int eig_batch_set(eig_batch_t b, int32_t knob, int32_t value) {
  if (!b) return EIG_EINVAL;
  switch (knob) {
    case EIG_KNOB_ROOTSOLVE:
      if (value != EIG_AUTO && value != EIG_ROOTSOLVE_GROUPED && value != EIG_ROOTSOLVE_PERSISTENT)
        return EIG_EINVAL;
      b->force_root = value;
      return EIG_OK;
    case EIG_KNOB_GEMM_TILE:
      if (value != EIG_AUTO && value != 64 && value != 128) return EIG_EINVAL;
      b->force_tile = value;
      return EIG_OK;
    case EIG_KNOB_GRAPHS:
      if (value != 0 && value != 1) return EIG_EINVAL;
      b->use_graphs = value;
      return EIG_OK;
    default:
      return EIG_EINVAL;
  }
}

int eig_batch_get(eig_batch_t b, int32_t knob, int64_t* value) {
  if (!b || !value) return EIG_EINVAL;
  switch (knob) {
    case EIG_KNOB_ROOTSOLVE: *value = b->last_root; return EIG_OK;
    case EIG_KNOB_GEMM_TILE: *value = b->last_tile; return EIG_OK;
    case EIG_KNOB_GRAPHS: *value = b->last_graph; return EIG_OK;
    case EIG_STAT_GRAPH_LAUNCHES: *value = b->graph_launches; return EIG_OK;
    case EIG_STAT_GRAPHS_CACHED: {
      long long c = 0;
      for (auto& kv : b->graphs) c += kv.second.exec ? 1 : 0;
      *value = c;
      return EIG_OK;
    }
    default: return EIG_EINVAL;
  }
}

int eig_update_batch(eig_batch_t b, const eig_batch_item* items, int32_t count, uint32_t mode,
                     void* hip_stream) {
  TraceRange trace("eig_update_batch");
  if (!b || !items || count < 1 || count > b->max_items) return EIG_EINVAL;
  if (mode & ~(uint32_t)(EIG_VALUES_ONLY | EIG_QW_FARFIELD)) return EIG_EUNSUPPORTED;
  const bool vo = (mode & EIG_VALUES_ONLY) != 0;
  const bool want_ff = (mode & EIG_QW_FARFIELD) && !vo;
  // argument checks (nothing is enqueued if one fails)
  std::vector<int> masks(count);
  for (int i = 0; i < count; ++i) {
    const eig_batch_item& it = items[i];
    eig_state_s* s = it.state;
    if (!s || !it.K || it.k < 1 || it.ldk < s->n) return EIG_EINVAL;
    if (it.k > EIG_KMAX) return EIG_EUNSUPPORTED;
    if (it.k > s->n || s->n > (int64_t)1 << 30) return EIG_EINVAL;
    if (s->device != b->device) return EIG_EINVAL;
    if (!s->uploaded) return EIG_ESTATE;
    int m = 0;
    for (int c = 0; c < it.k; ++c) {
      if (it.sigma[c] == 1)
        m |= 1 << c;
      else if (it.sigma[c] != -1)
        return EIG_EINVAL;
    }
    masks[i] = m;
    for (int j = 0; j < i; ++j)
      if (items[j].state == s) return EIG_EINVAL;  // one update per state per batch
  }
  DeviceGuard g(b->device);
  if (!g.ok) return EIG_EDEVICE;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);

  // plan: order, class offsets, block counts, shape key
  Plan p;
  p.count = count;
  p.order.resize(count);
  for (int i = 0; i < count; ++i) p.order[i] = i;
  std::stable_sort(p.order.begin(), p.order.end(), [&](int a, int c) {
    if (items[a].k != items[c].k) return items[a].k < items[c].k;
    return items[a].state->n > items[c].state->n;
  });
  for (int i = 0; i < count; ++i) p.cnt[items[i].k] += 1;
  for (int k = 1, acc = 0; k <= KMAX; ++k) {
    p.off[k] = acc;
    acc += p.cnt[k];
  }
  p.key = vo ? "v" : (want_ff ? "F" : "f");
  char buf[48];
  for (int pos = 0; pos < count; ++pos) {
    const eig_batch_item& it = items[p.order[pos]];
    snprintf(buf, sizeof buf, "|%d,%lld", (int)it.k, (long long)it.state->n);
    p.key += buf;
  }

  // tuning choices for this shape
  eig_batch_s::Tune& tu = b->tune[p.key];
  int root_form, tile;
  bool measuring = false;
  if (tu.done) {
    root_form = tu.root;
    tile = tu.tile;
  } else {
    root_form = (tu.phase == 0) ? EIG_ROOTSOLVE_GROUPED : EIG_ROOTSOLVE_PERSISTENT;
    tile = (tu.phase == 0) ? 128 : 64;
    measuring = true;
  }
  if (b->force_root != EIG_AUTO) root_form = b->force_root;
  if (b->force_tile != EIG_AUTO) tile = b->force_tile;
  if (b->force_root != EIG_AUTO && (vo || b->force_tile != EIG_AUTO)) measuring = false;

  // far-field instances: their buffers (sized for rank EIG_KMAX, so that later
  // batches of other ranks do not reallocate them), allocated on first use
  p.ff.assign(count, 0);
  p.host_works.resize(count);
  p.states.resize(count);
  for (int pos = 0; pos < count; ++pos) {
    const eig_batch_item& it = items[p.order[pos]];
    eig_state_s* s = it.state;
    if (!want_ff || !ff_eligible((int)s->n, (int)it.k)) continue;
    const size_t need = ff_bytes_max((int)s->n);
    if (s->ff_bytes < need) {
      if (s->ff_block) {
        HIPCHK(hipDeviceSynchronize());
        (void)hipFree(s->ff_block);
        s->ff_block = nullptr;
        s->ff_bytes = 0;
      }
      if (hipMalloc(&s->ff_block, need) != hipSuccess) {
        (void)hipGetLastError();
        s->ff_block = nullptr;
        return EIG_ENOMEM;
      }
      s->ff_bytes = need;
    }
    p.ff[pos] = 1;
    p.any_ff = true;
  }

  // per-call descriptors into a pinned slot
  layout(p);
  const int sl = b->slot;
  b->slot ^= 1;
  HIPCHK(hipEventSynchronize(b->slot_ev[sl]));
  char* h = static_cast<char*>(b->h_slot[sl]);
  Work* hw = reinterpret_cast<Work*>(h);
  GemmDesc* hg = reinterpret_cast<GemmDesc*>(h + p.gemm_bytes_off);
  int* hp = reinterpret_cast<int*>(h + p.prefix_bytes_off);
  int run[KMAX + 1][NKIND] = {};
  for (int pos = 0; pos < count; ++pos) {
    const eig_batch_item& it = items[p.order[pos]];
    eig_state_s* s = it.state;
    const int k = (int)it.k, n = (int)s->n;
    hw[pos] = make_work(s, k, it.K, (int)it.ldk, masks[p.order[pos]], vo);
    p.host_works[pos] = hw[pos];
    p.states[pos] = s;
    const int local = pos - p.off[k];
    const bool ff = p.ff[pos] != 0;  // W and Q' by its own far-field launches
    const int nb[NKIND] = {qtk_blocks(n, k), root_blocks(n), ff ? 0 : wbuild_blocks(n),
                           ff ? 0 : reflect_blocks(n), solve_blocks(n, k)};
    for (int kind = 0; kind < NKIND; ++kind) {
      int* pre = hp + p.poff[k][kind];
      pre[local] = run[k][kind];
      run[k][kind] += nb[kind];
      pre[local + 1] = run[k][kind];
    }
  }
  for (int k = 1; k <= KMAX; ++k)
    for (int kind = 0; kind < NKIND; ++kind) p.blocks[k][kind] = run[k][kind];
  // GEMM: instances in the same order (n descending within each k)
  int* gp = hp + p.gemm_poff;
  gp[0] = 0;
  for (int pos = 0; pos < count; ++pos) {
    const Work& w = hw[pos];
    GemmDesc d;
    d.A = w.Q_in;
    d.B = w.W;
    d.C = w.Q_out;
    d.status = &w.st->status;
    d.n = w.n;
    d.vec = !(w.n & 1);
    hg[pos] = d;
    gp[pos + 1] = gp[pos] + (p.ff[pos] ? 0 : gemm_tiles(w.n, tile));
  }
  p.gemm_blocks = gp[count];
  HIPCHK(hipMemcpyAsync(b->d_block, h, p.bytes, hipMemcpyHostToDevice, st));
  HIPCHK(hipEventRecord(b->slot_ev[sl], st));

  b->last_root = root_form;
  b->last_tile = vo ? 0 : tile;
  b->last_graph = 0;
  if (measuring) {
    HIPCHK(enqueue(b, p, vo, root_form, tile, st, b->tev));
    HIPCHK(hipEventSynchronize(vo ? b->tev[1] : b->tev[3]));
    float rms = 0.0f, gms = 0.0f;
    HIPCHK(hipEventElapsedTime(&rms, b->tev[0], b->tev[1]));
    if (!vo) HIPCHK(hipEventElapsedTime(&gms, b->tev[2], b->tev[3]));
    const int ph = tu.phase;
    tu.root_ms[ph] = rms;
    tu.gemm_ms[ph] = gms;
    tu.phase += 1;
    if (tu.phase == 2) {
      tu.root = (tu.root_ms[1] < tu.root_ms[0]) ? EIG_ROOTSOLVE_PERSISTENT : EIG_ROOTSOLVE_GROUPED;
      tu.tile = (!vo && tu.gemm_ms[1] < tu.gemm_ms[0]) ? 64 : 128;
      tu.done = true;
    }
  } else if (b->use_graphs && !p.any_ff) {
    // (a batch with far-field instances is launched directly: its far-field
    // launches take each state's buffers as arguments, which a replay for other
    // states of the same shape would reuse)
    snprintf(buf, sizeof buf, "#%d,%d", root_form, tile);
    const std::string gkey = p.key + buf;
    eig_batch_s::Entry& en = b->graphs[gkey];
    en.seen += 1;
    if (!en.exec && en.seen >= 2) {
      if ((int)b->graphs.size() > MAX_GRAPHS) {
        // keep the cache bounded: drop every other entry's graph
        for (auto& kv : b->graphs)
          if (kv.first != gkey && kv.second.exec) {
            (void)hipGraphExecDestroy(kv.second.exec);
            kv.second.exec = nullptr;
          }
      }
      hipGraph_t graph = nullptr;
      HIPCHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
      const hipError_t e1 = enqueue(b, p, vo, root_form, tile, b->cap, nullptr);
      const hipError_t e2 = hipStreamEndCapture(b->cap, &graph);
      if (e1 != hipSuccess || e2 != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        return EIG_EDEVICE;
      }
      const hipError_t e3 = hipGraphInstantiate(&en.exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e3 != hipSuccess) {
        en.exec = nullptr;
        return EIG_EDEVICE;
      }
    }
    if (en.exec) {
      HIPCHK(hipGraphLaunch(en.exec, st));
      b->last_graph = 1;
      b->graph_launches += 1;
    } else {
      HIPCHK(enqueue(b, p, vo, root_form, tile, st, nullptr));
    }
  } else {
    HIPCHK(enqueue(b, p, vo, root_form, tile, st, nullptr));
  }

  // host bookkeeping of the states
  for (int i = 0; i < count; ++i) {
    eig_state_s* s = items[i].state;
    s->last_k = (int)items[i].k;
    s->last_p = __builtin_popcount((unsigned)masks[i]);
    s->last_q = s->last_k - s->last_p;
    s->timed = false;
    s->last_vo = vo;
    if (!vo) s->enq_gen += 1;
  }
  return EIG_OK;
}

}  // extern "C"
