// Solver context shared by the translation units of the C ABI.
#pragma once
#include <stdint.h>

#include <vector>

#include "../../include/fmm355.h"
#include "common.h"

struct fmm_ctx {
  fmm_params prm;
  int64_t max_n;
  hipStream_t stream;
  hipStream_t side;        // library-owned second stream (P2P beside the multipole passes)
  hipEvent_t fork, join;
  int device;
  DevTree t;
  std::vector<void *> allocs;
  // host copy of the last build
  Header hh;
  bool tree_valid;
  std::vector<fmm_request> b_reqs;  // requests of the last build
  int64_t b_n;                      // their active particles in all
  double b_eps, b_theta;
  // request table uploads: a ring of pinned staging slots (each reused only
  // after the copy from it has completed) and the last table sent, so an
  // unchanged table is not sent again
  static constexpr int UP_SLOTS = 8;
  char *up_pin[UP_SLOTS];
  hipEvent_t up_ev[UP_SLOTS];
  bool up_ev_set[UP_SLOTS];
  int up_next;
  size_t up_bytes;                  // bytes of one slot = device request region
  std::vector<char> up_last;
  bool up_valid;
  Header *pin_hdr;                  // pinned destination of header readbacks
  hipEvent_t hdr_ev;                // recorded after a queued header readback
  hipEvent_t up_done;               // upward pass queued beside the walk has finished
  int n_nodes, depth;
  int small_max;           // single-workgroup build and walk for batches of at most this many particles
  // split levels of recent multi-workgroup builds: the next build queues the
  // tree and the walk for the deepest of them behind the sort, with one
  // readback at the end, and falls back to reading the split depth first when
  // its tree needed more levels
  static constexpr int LEVEL_HIST = 4;
  int lvl_hist[LEVEL_HIST];
  int lvl_hist_n;
  bool predict_levels;
  // integrator
  hhs_run *own_run;       // scratch of hhs_init / hhs_step (one system)
  int32_t *split_cnt;     // [cap_split] fast-set sizes of pending splits
  int cap_split;
  int32_t *pin_split;     // [cap_split] pinned destination of split-count readbacks
  double *inv_part;
  double *dvec;            // [3][max_n] sorted source vectors of the vector-source pass
                           // (allocated by its first call)
  double *gstage;          // [6][max_n] near part of the force gradient in sorted order
                           // (allocated by the first fmm_forces_grad)
  int64_t stat_calls, stat_parts, stat_builds;
  PhaseTimer timer;
  char err[512];
};


fmm_status fmm_fail(fmm_ctx *c, fmm_status st, const char *fmt, ...);

template <typename T>
bool fmm_dalloc(fmm_ctx *c, T **p, int64_t count) {
  void *q = nullptr;
  size_t bytes = (size_t)(count > 1 ? count : 1) * sizeof(T);
  if (hipMalloc(&q, bytes) != hipSuccess) return false;
  c->allocs.push_back(q);
  *p = (T *)q;
  return true;
}
void fmm_dfree(fmm_ctx *c, void *p);
