// state.h -- the host-side state object behind eig_state_t (shared by the
// single-update and the batched entry points).
#pragma once

#include "eigupd.h"
#include "internal.h"

struct eig_state_s {
  int device = 0;
  int64_t n = 0;
  bool lean = false;      // Q[], W not owned: lent per update (serving)
  void* block = nullptr;
  size_t block_bytes = 0;
  double* lam[2] = {nullptr, nullptr};
  double* Q[2] = {nullptr, nullptr};
  double* lam_vo = nullptr;
  double* lam_x = nullptr;   // eigenvalues between the chained parts of a rank > 8 update
  double* Kbuf = nullptr;    // n x EIG_KMAX_GENERIC: host K of EIG_HOST_INPUT
  void* lp_block = nullptr;  // slice planes of the reduced-precision modes (lazily)
  size_t lp_bytes = 0;
  void* ff_block = nullptr;  // buffers of the far-field product (lazily)
  size_t ff_bytes = 0;
  double* Q_x = nullptr;     // n x n: Q between the chained parts of a rank > 8 update (lazily)
  eigupd::Work w{};       // workspace pointers (carved from block)
  hipEvent_t ev[9] = {};  // phase events (EIG_PHASE_TIMING)
  bool timed = false;
  int64_t enq_gen = 0;    // updates enqueued since upload (selects the buffer)
  bool uploaded = false;  // a decomposition has been uploaded
  bool last_vo = false;   // the last update was values-only
  int last_k = 0;         // rank of the last update
  int last_p = 0, last_q = 0;  // its numbers of sigma_c = +1 and -1
};

namespace eigupd {

// Lays out the O(n) workspace of one update of order n (U, deflation, reduced
// problem, roots, column parameters, status and info) at base + off, each
// buffer 256-byte aligned; base == nullptr is a sizing pass that leaves the
// pointers null.  Returns the offset just past the last buffer.
size_t carve_workspace(Work& w, size_t n, char* base, size_t off);

// Creates a state; lean: without its own Q buffers and W (24 n^2 bytes fewer),
// for an owner that lends them per update.
int state_create(eig_state_t* out, int64_t n, int32_t device, bool lean);

// Descriptor of one update of state s (rank k, device K with leading
// dimension ldk, bit c of sig_pos_mask set <=> sigma_c = +1).  Reads the
// buffer that holds the last enqueued decomposition and writes the other.
inline Work make_work(const eig_state_s* s, int k, const double* K, int ldk, int sig_pos_mask,
                      bool values_only) {
  Work w = s->w;
  w.k = k;
  w.sig_pos_mask = sig_pos_mask;
  w.K = K;
  w.ldk = ldk;
  const int cur = (int)(s->enq_gen & 1);
  w.lam_in = s->lam[cur];
  w.Q_in = s->Q[cur];
  w.lam_out = s->lam[cur ^ 1];
  w.Q_out = s->Q[cur ^ 1];
  w.lam_fin = values_only ? s->lam_vo : w.lam_out;
  return w;
}

}  // namespace eigupd
