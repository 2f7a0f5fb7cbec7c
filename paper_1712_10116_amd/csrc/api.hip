// Host side of the C ABI declared in include/fmm355.h.
//
// A context owns one device workspace sized from max_n at creation.  Every
// call is queued on the context's stream; fmm_build waits once, at its end,
// to read the list sizes (and to regrow a list buffer that turned out too
// small, which is then rebuilt once).
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "../../include/fmm355.h"
#include "common.h"
#include "context.h"
#include "hhs_kernels.h"

static PhaseTimer *timer_of(fmm_ctx *c) { return c->timer.on ? &c->timer : nullptr; }

fmm_status fmm_fail(fmm_ctx *c, fmm_status st, const char *fmt, ...) {
  if (c) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->err, sizeof(c->err), fmt, ap);
    va_end(ap);
  }
  return st;
}

#define HIPCHK(c, call)                                                                       \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail((c), FMM_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));          \
  } while (0)

static int coeffs(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

#define fail fmm_fail
#define dalloc fmm_dalloc
#define dfree fmm_dfree

void fmm_dfree(fmm_ctx *c, void *p) {
  if (!p) return;
  auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
  if (it != c->allocs.end()) c->allocs.erase(it);
  (void)hipFree(p);
}

// node-sized arrays
static bool alloc_nodes(fmm_ctx *c, int64_t cap) {
  DevTree &t = c->t;
  if (cap >= ((int64_t)1 << 28)) return false;  // node ids carry a 3-bit tag in the walk
  t.cap_nodes = cap;
  size_t real = c->prm.precision == FMM_PREC_MIXED ? sizeof(float) : sizeof(double);
  bool ok = dalloc(c, &t.nbeg, cap) && dalloc(c, &t.nend, cap) && dalloc(c, &t.nlev, cap) &&
            dalloc(c, &t.nparent, cap) && dalloc(c, &t.nchild0, cap) &&
            dalloc(c, &t.nnchild, cap) && dalloc(c, &t.ngeo, cap) &&
            dalloc(c, &t.bounds, cap * 8) && dalloc(c, &t.m2l_off, cap) &&
            dalloc(c, &t.m2l_cnt, cap) && dalloc(c, &t.p2p_off, cap) &&
            dalloc(c, &t.p2p_cnt, cap) && dalloc(c, &t.open_off, cap) &&
            dalloc(c, &t.open_cnt, cap) && dalloc(c, &t.nreq, cap);
  if (!ok) return false;
  char *m = nullptr, *l = nullptr, *mh = nullptr;
  ok = dalloc(c, &m, (int64_t)(cap * t.kmax * real)) && dalloc(c, &l, (int64_t)(cap * t.kmax * real)) &&
       dalloc(c, &mh, (int64_t)(cap * t.khmax * real));
  t.M = m;
  t.L = l;
  t.Mh = mh;
  return ok;
}

static void free_nodes(fmm_ctx *c) {
  DevTree &t = c->t;
  void *ptrs[] = {t.nbeg, t.nend, t.nlev, t.nparent, t.nchild0, t.nnchild, t.ngeo, t.bounds,
                  t.m2l_off, t.m2l_cnt, t.p2p_off, t.p2p_cnt, t.open_off, t.open_cnt, t.M, t.L,
                  t.Mh, t.nreq};
  for (void *p : ptrs) dfree(c, p);
}

// Request-sized arrays (regrown when a batch holds more requests).  The
// request table, its particle offsets and its block offsets share one device
// region, mirrored by pinned host staging slots, so a table is sent in one copy.
static size_t req_region_bytes(int cap) {
  return sizeof(DevReq) * (size_t)cap + 2 * sizeof(int32_t) * (size_t)(cap + 1);
}

static bool alloc_reqs(fmm_ctx *c, int cap) {
  DevTree &t = c->t;
  for (int k = 0; k < fmm_ctx::UP_SLOTS; ++k)
    if (c->up_ev_set[k]) (void)hipEventSynchronize(c->up_ev[k]);
  void *ptrs[] = {t.reqs, t.box, t.bbox_part};
  for (void *p : ptrs) dfree(c, p);
  t.reqs = nullptr;
  t.cap_req = cap;
  const size_t bytes = req_region_bytes(cap);
  char *region = nullptr;
  if (!dalloc(c, &region, (int64_t)bytes) || !dalloc(c, &t.box, cap) ||
      !dalloc(c, &t.bbox_part, (int64_t)cap * FMM_BBOX_BLOCKS * 6))
    return false;
  t.reqs = (DevReq *)region;
  t.req_off = (int32_t *)(region + sizeof(DevReq) * (size_t)cap);
  t.blk_off = t.req_off + cap + 1;
  for (int k = 0; k < fmm_ctx::UP_SLOTS; ++k) {
    if (c->up_pin[k]) (void)hipHostFree(c->up_pin[k]);
    c->up_pin[k] = nullptr;
    if (hipHostMalloc((void **)&c->up_pin[k], bytes) != hipSuccess) return false;
  }
  c->up_bytes = bytes;
  c->up_valid = false;
  return true;
}

extern "C" fmm_status fmm_create(const fmm_params *prm, int64_t max_n, void *stream,
                                 fmm_ctx **out) {
  if (!prm || !out) return FMM_EINVAL;
  *out = nullptr;
  if (max_n < 1 || max_n > (int64_t)1 << 30) return FMM_EINVAL;
  if (prm->p_max < 1 || prm->p_max > 8 || prm->leaf_size < 1 || prm->leaf_size > 4096 ||
      (prm->kernel != FMM_KERNEL_WENDLAND_C2 && prm->kernel != FMM_KERNEL_PLUMMER) ||
      (prm->precision != FMM_PREC_FP64 && prm->precision != FMM_PREC_MIXED))
    return FMM_EINVAL;
  fmm_ctx *c = new (std::nothrow) fmm_ctx();
  if (!c) return FMM_ENOMEM;
  c->prm = *prm;
  c->max_n = max_n;
  c->small_max = SMALL_AUTO_N;
  c->predict_levels = false;
  c->lvl_hist_n = 0;
  c->stream = (hipStream_t)stream;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return FMM_EDEVICE;
  }
  DevTree &t = c->t;
  memset(&t, 0, sizeof(t));
  bool pins = hipHostMalloc((void **)&c->pin_hdr, sizeof(Header)) == hipSuccess &&
              hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&c->join, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&c->hdr_ev, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&c->up_done, hipEventDisableTiming) == hipSuccess;
  for (int k = 0; pins && k < fmm_ctx::UP_SLOTS; ++k)
    pins = hipEventCreateWithFlags(&c->up_ev[k], hipEventDisableTiming) == hipSuccess;
  if (!pins) {
    fmm_destroy(c);
    return FMM_ENOMEM;
  }
  t.kmax = coeffs(prm->p_max);
  t.khmax = (prm->p_max + 1) * (prm->p_max + 1);
  t.cap_n = max_n;
  int64_t n = max_n;
  int64_t cap_nodes = 8 * n / prm->leaf_size + 1024;
  // radix histograms: one column per tile, and for sorts of at most
  // SORT_RAW_TILES tiles one slice per pass
  const int64_t sort_tiles = (n + SORT_TILE - 1) / SORT_TILE;
  const int64_t sort_hist_n =
      256 * std::max<int64_t>(sort_tiles, SORT_MAX_PASSES * std::min<int64_t>(sort_tiles, SORT_RAW_TILES)) +
      256;
  bool ok = dalloc(c, &t.key, n) && dalloc(c, &t.key2, n) && dalloc(c, &t.slot, n) &&
            dalloc(c, &t.slot2, n) && dalloc(c, &t.sx, n) && dalloc(c, &t.sy, n) &&
            dalloc(c, &t.sz, n) && dalloc(c, &t.sm, n) && dalloc(c, &t.sm32, n) &&
            dalloc(c, &t.leaf_of, n) && dalloc(c, &t.near, 4 * n) && dalloc(c, &t.pak, n) &&
            dalloc(c, &t.scan_part, FMM_SCAN_BLOCKS) && dalloc(c, &t.slot_req, n) &&
            dalloc(c, &t.sort_hist, sort_hist_n) &&
            dalloc(c, &t.sort_dtot, 256) && dalloc(c, &t.scan_blk, n / 1024 + 64) &&
            dalloc(c, &t.hdr, 1) && alloc_reqs(c, 16) && alloc_nodes(c, cap_nodes);
  if (ok) {
    t.cap_m2l = 96 * cap_nodes;
    t.cap_p2p = 32 * cap_nodes;
    t.cap_open = 16 * cap_nodes;
    ok = dalloc(c, &t.m2l_src, t.cap_m2l) && dalloc(c, &t.p2p_src, t.cap_p2p) &&
         dalloc(c, &t.open_buf0, t.cap_open) && dalloc(c, &t.open_buf1, t.cap_open);
  }
  ok = ok && dalloc(c, &c->inv_part, FMM_INV_BLOCKS * 12);
  if (!ok) {
    fmm_destroy(c);
    return FMM_ENOMEM;
  }
  if (hipMemsetAsync(t.hdr, 0, sizeof(Header), c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    fmm_destroy(c);
    return FMM_EDEVICE;
  }
  *out = c;
  return FMM_OK;
}

extern "C" fmm_status fmm_destroy(fmm_ctx *c) {
  if (!c) return FMM_EINVAL;
  (void)hipStreamSynchronize(c->stream);
  if (c->timer.ready)
    for (int i = 0; i < PhaseTimer::CAP; ++i) {
      (void)hipEventDestroy(c->timer.a[i]);
      (void)hipEventDestroy(c->timer.b[i]);
    }
  if (c->own_run) hhs_run_destroy(c->own_run);
  for (void *p : c->allocs) (void)hipFree(p);
  for (int k = 0; k < fmm_ctx::UP_SLOTS; ++k) {
    if (c->up_pin[k]) (void)hipHostFree(c->up_pin[k]);
    if (c->up_ev[k]) (void)hipEventDestroy(c->up_ev[k]);
  }
  if (c->pin_hdr) (void)hipHostFree(c->pin_hdr);
  if (c->pin_split) (void)hipHostFree(c->pin_split);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
  }
  if (c->fork) (void)hipEventDestroy(c->fork);
  if (c->join) (void)hipEventDestroy(c->join);
  if (c->hdr_ev) (void)hipEventDestroy(c->hdr_ev);
  if (c->up_done) (void)hipEventDestroy(c->up_done);
  delete c;
  return FMM_OK;
}

extern "C" const char *fmm_last_error(const fmm_ctx *c) { return c ? c->err : "null context"; }

extern "C" fmm_status fmm_set_small_path(fmm_ctx *c, int enable) {
  if (!c || enable < 0 || enable > 2) return FMM_EINVAL;
  c->small_max = enable == 0 ? -1 : enable == 1 ? SMALL_AUTO_N : SMALL_N;
  return FMM_OK;
}

extern "C" fmm_status fmm_set_level_prediction(fmm_ctx *c, int enable) {
  if (!c) return FMM_EINVAL;
  c->predict_levels = enable != 0;
  c->lvl_hist_n = 0;
  return FMM_OK;
}

// split levels of the recent builds (0: none recorded)
static int predicted_levels(const fmm_ctx *c) {
  int m = 0;
  for (int i = 0; i < std::min(c->lvl_hist_n, fmm_ctx::LEVEL_HIST); ++i) m = std::max(m, c->lvl_hist[i]);
  return m;
}

static void record_levels(fmm_ctx *c, int levels) {
  c->lvl_hist[c->lvl_hist_n % fmm_ctx::LEVEL_HIST] = levels;
  c->lvl_hist_n++;
}

static fmm_status check_requests(fmm_ctx *c, int n_req, const fmm_request *reqs, bool eval,
                                 int64_t *n_all) {
  if (!c) return FMM_EINVAL;
  if (n_req < 1 || !reqs) return fail(c, FMM_EINVAL, "need at least one request");
  int64_t n = 0;
  for (int r = 0; r < n_req; ++r) {
    const fmm_request &q = reqs[r];
    if (q.n_active < 0 || q.n_total < 0 || q.n_total > (int64_t)INT32_MAX)
      return fail(c, FMM_EINVAL, "request %d: bad sizes", r);
    if (q.n_active > 0 && !q.active && q.n_total != q.n_active)
      return fail(c, FMM_EINVAL, "request %d: n_total=%lld inconsistent with n_active=%lld", r,
                  (long long)q.n_total, (long long)q.n_active);
    if (q.n_active > 0 && !q.pos) return fail(c, FMM_EINVAL, "request %d: pos is NULL", r);
    if (eval && q.n_active > 0 && q.mass && (!q.acc || !q.pot))
      return fail(c, FMM_EINVAL, "request %d: NULL acc/pot", r);
    n += q.n_active;
  }
  if (n > c->max_n)
    return fail(c, FMM_EINVAL, "%lld active particles exceed max_n=%lld", (long long)n,
                (long long)c->max_n);
  *n_all = n;
  return FMM_OK;
}

// Stage the request table in the next pinned slot and send it in one copy,
// unless it equals the table last sent.  Blocks per request for the box
// reduction: ceil(n / 2048), at least 1 and at most FMM_BBOX_BLOCKS.
static fmm_status upload_requests(fmm_ctx *c, int n_req, const fmm_request *reqs, int *n_blk) {
  DevTree &t = c->t;
  if (n_req > t.cap_req && !alloc_reqs(c, std::max(n_req, 2 * t.cap_req)))
    return fail(c, FMM_ENOMEM, "request table for %d requests", n_req);
  const int k = c->up_next;
  if (c->up_ev_set[k]) HIPCHK(c, hipEventSynchronize(c->up_ev[k]));
  char *stage = c->up_pin[k];
  memset(stage, 0, c->up_bytes);
  DevReq *hr = (DevReq *)stage;
  int32_t *ho = (int32_t *)(stage + sizeof(DevReq) * (size_t)t.cap_req);
  int32_t *hb = ho + t.cap_req + 1;
  int off = 0, blk = 0;
  for (int r = 0; r < n_req; ++r) {
    const fmm_request &q = reqs[r];
    hr[r].pos = q.pos;
    hr[r].active = q.active;
    hr[r].mass = q.mass;
    hr[r].acc = q.acc;
    hr[r].pot = q.pot;
    hr[r].sinks = q.sinks;
    hr[r].n_total = q.n_total;
    hr[r].off = off;
    hr[r].n = (int32_t)q.n_active;
    ho[r] = off;
    hb[r] = blk;
    off += (int)q.n_active;
    blk += (int)std::min<int64_t>(FMM_BBOX_BLOCKS, std::max<int64_t>(1, (q.n_active + 2047) / 2048));
  }
  ho[n_req] = off;
  hb[n_req] = blk;
  t.n_req = n_req;
  if (!(c->up_valid && c->up_last.size() == c->up_bytes &&
        memcmp(c->up_last.data(), stage, c->up_bytes) == 0)) {
    HIPCHK(c, hipMemcpyAsync(t.reqs, stage, c->up_bytes, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipEventRecord(c->up_ev[k], c->stream));
    c->up_ev_set[k] = true;
    c->up_next = (k + 1) % fmm_ctx::UP_SLOTS;
    c->up_last.assign(stage, stage + c->up_bytes);
    c->up_valid = true;
  }
  if (n_blk) *n_blk = blk;
  return FMM_OK;
}

// header readback through pinned memory; waits for the stream
static fmm_status read_header(fmm_ctx *c) {
  HIPCHK(c, hipMemcpyAsync(c->pin_hdr, c->t.hdr, sizeof(Header), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  memcpy(&c->hh, c->pin_hdr, sizeof(Header));
  return FMM_OK;
}

// Regrow the list buffer that overflowed.  A walk that overflows stops
// writing, so `need` (the entries it tried to place) can undercount what the
// whole walk needs: the capacity at least doubles each time.
static fmm_status regrow_lists(fmm_ctx *c, int which, int64_t need) {
  DevTree &t = c->t;
  const int64_t old = which == OVF_M2L ? t.cap_m2l : which == OVF_P2P ? t.cap_p2p : t.cap_open;
  int64_t cap = std::max(need + need / 4 + 1024, 2 * old);
  if (which == OVF_M2L) {
    dfree(c, t.m2l_src);
    t.m2l_src = nullptr;
    if (!dalloc(c, &t.m2l_src, cap)) return fail(c, FMM_ENOMEM, "M2L list regrow failed");
    t.cap_m2l = cap;
  } else if (which == OVF_P2P) {
    dfree(c, t.p2p_src);
    t.p2p_src = nullptr;
    if (!dalloc(c, &t.p2p_src, cap)) return fail(c, FMM_ENOMEM, "P2P list regrow failed");
    t.cap_p2p = cap;
  } else {
    dfree(c, t.open_buf0);
    dfree(c, t.open_buf1);
    t.open_buf0 = t.open_buf1 = nullptr;
    if (!dalloc(c, &t.open_buf0, cap) || !dalloc(c, &t.open_buf1, cap))
      return fail(c, FMM_ENOMEM, "open list regrow failed");
    t.cap_open = cap;
  }
  return FMM_OK;
}

static void set_eval_args(fmm_ctx *c, EvalArgs &e, int64_t n_all, int p, double eps) {
  e.n = (int)n_all;
  e.p = p;
  e.kernel = c->prm.kernel;
  e.mixed = c->prm.precision == FMM_PREC_MIXED;
  e.eps = eps;
  e.tm = timer_of(c);
  e.side = c->side;
  e.fork = c->fork;
  e.join = c->join;
}

static void count_evaluation(fmm_ctx *c, int n_req, const fmm_request *reqs) {
  c->stat_calls++;
  for (int r = 0; r < n_req; ++r)
    if (reqs[r].mass) c->stat_parts += reqs[r].n_active;
}

// Build (and, with p_fused > 0, evaluate at order p_fused): when the
// predicted sequence runs, the evaluation is queued behind the walk before the
// host reads the tree header, with the tree's sizes taken on the device; if
// the header then shows that the prediction fell short or a workspace
// overflowed, the build is redone the classic way and *evaluated stays false
// (the caller evaluates again, overwriting whatever the queued kernels wrote).
static fmm_status build_impl(fmm_ctx *c, int n_req, const fmm_request *reqs, double eps,
                             double theta, int p_fused, bool *evaluated, bool *upward) {
  int64_t n_all = 0;
  fmm_status st = check_requests(c, n_req, reqs, p_fused > 0, &n_all);
  if (st != FMM_OK) return st;
  if (!(theta > 0.0) || !(eps >= 0.0) || !std::isfinite(theta) || !std::isfinite(eps))
    return fail(c, FMM_EINVAL, "need theta > 0 and eps >= 0");
  c->tree_valid = false;
  int n_blk = 0;
  st = upload_requests(c, n_req, reqs, &n_blk);
  if (st != FMM_OK) return st;
  BuildArgs a = {};
  a.n = (int)n_all;
  a.n_req = n_req;
  a.n_blk = n_blk;
  a.leaf_size = c->prm.leaf_size;
  a.eps = eps;
  a.theta = theta;
  a.tm = timer_of(c);
  auto finish = [&](int depth) {
    c->n_nodes = c->hh.lvl_start[FMM_NLEVELS];
    c->depth = depth;
    c->tree_valid = true;
    c->b_reqs.assign(reqs, reqs + n_req);
    c->b_n = n_all;
    c->b_eps = eps;
    c->b_theta = theta;
    c->stat_builds++;
    return FMM_OK;
  };
  auto tree_depth = [&]() {
    int depth = 0;
    for (int l = 0; l < FMM_NLEVELS; ++l)
      if (c->hh.lvl_start[l + 1] > c->hh.lvl_start[l]) depth = l;
    return depth;
  };
  // 0. small batches: build and walk in two single-workgroup launches and one
  // readback; anything that needs more room falls through to the general path
  if (n_all <= c->small_max) {
    HIPCHK(c, launch_build_small(c->t, a, c->stream));
    HIPCHK(c, launch_traverse_small(c->t, a, c->stream));
    st = read_header(c);
    if (st != FMM_OK) return st;
    if (c->hh.nonfinite) return fail(c, FMM_ENONFINITE, "non-finite input position");
    if (c->hh.overflow & OVF_STACK) return fail(c, FMM_EOVERFLOW, "walk descent stack overflow");
    if (!(c->hh.overflow & (OVF_NODES | OVF_M2L | OVF_P2P | OVF_OPEN))) return finish(tree_depth());
  }
  // 1a. split levels predicted from recent builds: tree and walk queued behind
  // the sort, one readback.  The tree equals the one built below whenever the
  // prediction covers the split depth (levels past it split nothing); if it
  // does not, or a workspace overflowed, the classic sequence runs.
  const int pred = c->predict_levels ? predicted_levels(c) : 0;
  if (pred > 0) {
    int32_t prev[FMM_NLEVELS + 2];  // level starts of the last tree: grid estimates
    memcpy(prev, c->hh.lvl_start, sizeof(prev));
    const int prev_nodes = c->n_nodes;
    // the evaluation's grids come from the last tree: only for a batch of
    // the same systems within a quarter of its size
    const bool fuse = p_fused > 0 && n_req == (int)c->b_reqs.size() && 4 * n_all >= 3 * c->b_n &&
                      4 * n_all <= 5 * c->b_n;
    HIPCHK(c, launch_sort(c->t, a, c->stream));
    if (build_tree_direct_ok(a.leaf_size))
      HIPCHK(c, launch_build_tree_direct(c->t, a, pred, c->stream));
    else
      HIPCHK(c, launch_build_tree(c->t, a, pred, c->stream));
    if (fuse) {  // mass gather, P2M and M2M on the second stream, beside the walk
      EvalArgs u = {};
      set_eval_args(c, u, n_all, p_fused, eps);
      u.n_nodes = std::max(prev_nodes, 1);
      u.lvl_start_host = prev;
      u.depth = pred;
      u.dev = true;
      HIPCHK(c, hipEventRecord(c->fork, c->stream));
      HIPCHK(c, hipStreamWaitEvent(c->side, c->fork, 0));
      HIPCHK(c, launch_upward(c->t, u, c->side));
      HIPCHK(c, hipEventRecord(c->up_done, c->side));
    }
    HIPCHK(c, launch_traverse_dev(c->t, a, pred, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->pin_hdr, c->t.hdr, sizeof(Header), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipEventRecord(c->hdr_ev, c->stream));
    if (fuse) {
      EvalArgs e = {};
      set_eval_args(c, e, n_all, p_fused, eps);
      e.n_nodes = std::max(prev_nodes, 1);
      e.lvl_start_host = prev;
      e.depth = pred;
      e.dev = true;
      e.upward_done = true;
      e.up_done = c->up_done;
      HIPCHK(c, launch_evaluate(c->t, e, c->stream));
    }
    HIPCHK(c, hipEventSynchronize(c->hdr_ev));
    memcpy(&c->hh, c->pin_hdr, sizeof(Header));
    if (c->hh.nonfinite) return fail(c, FMM_ENONFINITE, "non-finite input position");
    const int need = std::min(FMM_MAXLEVEL, c->hh.max_prefix + 1);
    if (need <= pred &&
        !(c->hh.overflow & (OVF_NODES | OVF_M2L | OVF_P2P | OVF_OPEN | OVF_STACK | OVF_DEPTH))) {
      record_levels(c, need);
      st = finish(tree_depth());
      if (st == FMM_OK && fuse) {
        count_evaluation(c, n_req, reqs);
        *evaluated = true;
      }
      return st;
    }
  }
  // 1. tree; one readback of the level sizes (exact launches for the walk).
  // With the direct build the split depth need not be read first.
  int max_level = 0;
  const bool direct = build_tree_direct_ok(a.leaf_size);
  for (int attempt = 0;; ++attempt) {
    if (attempt == 4) return fail(c, FMM_EOVERFLOW, "node workspace still too small");
    HIPCHK(c, launch_sort(c->t, a, c->stream));
    if (direct) HIPCHK(c, launch_build_tree_direct(c->t, a, FMM_MAXLEVEL, c->stream));
    st = read_header(c);
    if (st != FMM_OK) return st;
    if (c->hh.nonfinite) return fail(c, FMM_ENONFINITE, "non-finite input position");
    // no cell below level split_depth + 1 holds more than leaf_size particles
    max_level = std::min(FMM_MAXLEVEL, c->hh.max_prefix + 1);
    if (!direct && !(c->hh.overflow & OVF_NODES)) {
      HIPCHK(c, launch_build_tree(c->t, a, max_level, c->stream));
      st = read_header(c);
      if (st != FMM_OK) return st;
    }
    if (!(c->hh.overflow & OVF_NODES)) break;
    int64_t need = std::max<int64_t>(std::max<int64_t>((int64_t)c->hh.lvl_start[FMM_NLEVELS],
                                                       n_req),
                                     2 * c->t.cap_nodes);
    free_nodes(c);
    if (!alloc_nodes(c, need + need / 4))
      return fail(c, FMM_ENOMEM, "node workspace regrow to %lld failed", (long long)need);
  }
  const int depth = tree_depth();
  int32_t lvl[FMM_NLEVELS + 2];
  memcpy(lvl, c->hh.lvl_start, sizeof(lvl));
  a.lvl_host = lvl;
  a.depth = depth;
  // with the masses known (fmm_forces), the mass gather, P2M and M2M need only
  // the tree: they run on the second stream beside the walk, which leaves
  // most of the chip idle
  bool up = false;
  if (p_fused > 0 && n_all > 0) {
    EvalArgs u = {};
    set_eval_args(c, u, n_all, p_fused, eps);
    u.n_nodes = lvl[FMM_NLEVELS];
    u.lvl_start_host = lvl;
    u.depth = depth;
    HIPCHK(c, hipEventRecord(c->fork, c->stream));
    HIPCHK(c, hipStreamWaitEvent(c->side, c->fork, 0));
    HIPCHK(c, launch_upward(c->t, u, c->side));
    HIPCHK(c, hipEventRecord(c->up_done, c->side));
    up = true;
  }
  // 2. symmetric walk; regrow a list buffer that turned out too small.  With
  // the masses known the evaluation is queued behind the first walk before the
  // header is read (no host round trip between them): its kernels take the
  // node count and level bounds from the header and do nothing if a list
  // buffer overflowed; then the lists are regrown, the walk is redone and
  // *evaluated stays false (the caller evaluates again).
  for (int attempt = 0; attempt < 10; ++attempt) {
    HIPCHK(c, launch_traverse(c->t, a, c->stream));
    bool queued = false;
    if (up && evaluated && attempt == 0) {
      // the header copy goes behind the walk, the evaluation behind it; the
      // host waits for the copy only
      HIPCHK(c, hipMemcpyAsync(c->pin_hdr, c->t.hdr, sizeof(Header), hipMemcpyDeviceToHost,
                               c->stream));
      HIPCHK(c, hipEventRecord(c->hdr_ev, c->stream));
      EvalArgs e = {};
      set_eval_args(c, e, n_all, p_fused, eps);
      e.n_nodes = lvl[FMM_NLEVELS];
      e.lvl_start_host = lvl;
      e.depth = depth;
      e.dev = true;
      e.exact = true;
      e.upward_done = true;
      e.up_done = c->up_done;
      HIPCHK(c, launch_evaluate(c->t, e, c->stream));
      queued = true;
      HIPCHK(c, hipEventSynchronize(c->hdr_ev));
      memcpy(&c->hh, c->pin_hdr, sizeof(Header));
    } else {
      st = read_header(c);
      if (st != FMM_OK) return st;
    }
    const Header &h = c->hh;
    if (h.overflow & OVF_STACK) return fail(c, FMM_EOVERFLOW, "walk descent stack overflow");
    if (h.overflow & (OVF_M2L | OVF_P2P | OVF_OPEN)) {
      if (h.overflow & OVF_M2L) {
        st = regrow_lists(c, OVF_M2L, h.m2l_cursor);
        if (st != FMM_OK) return st;
      }
      if (h.overflow & OVF_P2P) {
        st = regrow_lists(c, OVF_P2P, h.p2p_cursor);
        if (st != FMM_OK) return st;
      }
      if (h.overflow & OVF_OPEN) {
        uint32_t mx = 0;
        for (int l = 0; l < FMM_NLEVELS; ++l) mx = std::max(mx, h.open_cursor[l]);
        st = regrow_lists(c, OVF_OPEN, mx);
        if (st != FMM_OK) return st;
      }
      continue;
    }
    record_levels(c, max_level);
    st = finish(depth);
    if (st == FMM_OK && upward) *upward = up;
    if (st == FMM_OK && queued) {
      count_evaluation(c, n_req, reqs);
      *evaluated = true;
    }
    return st;
  }
  return fail(c, FMM_EOVERFLOW, "list workspace still too small after regrowth");
}

extern "C" fmm_status fmm_build_batched(fmm_ctx *c, int n_req, const fmm_request *reqs,
                                        double eps, double theta) {
  return build_impl(c, n_req, reqs, eps, theta, 0, nullptr, nullptr);
}

static fmm_status evaluate_impl(fmm_ctx *c, int n_req, const fmm_request *reqs, int p,
                                bool upward_done);

extern "C" fmm_status fmm_evaluate_batched(fmm_ctx *c, int n_req, const fmm_request *reqs, int p) {
  return evaluate_impl(c, n_req, reqs, p, false);
}

// upward_done: the build of these requests already queued the mass gather,
// P2M and M2M (build_impl with p_fused = p)
static fmm_status evaluate_impl(fmm_ctx *c, int n_req, const fmm_request *reqs, int p,
                                bool upward_done) {
  int64_t n_all = 0;
  fmm_status st = check_requests(c, n_req, reqs, true, &n_all);
  if (st != FMM_OK) return st;
  bool same = c->tree_valid && n_req == (int)c->b_reqs.size();
  for (int r = 0; same && r < n_req; ++r) {
    const fmm_request &a = reqs[r], &b = c->b_reqs[r];
    same = a.pos == b.pos && a.active == b.active && a.n_active == b.n_active &&
           a.n_total == b.n_total;
  }
  if (!same) return fail(c, FMM_ESTALE, "no tree built for these particles");
  if (p < 1 || p > c->prm.p_max || !eval_order_supported(p))
    return fail(c, FMM_EINVAL, "order p=%d unsupported (1..%d)", p, std::min(c->prm.p_max, 6));
  st = upload_requests(c, n_req, reqs, nullptr);
  if (st != FMM_OK) return st;
  EvalArgs e = {};
  set_eval_args(c, e, n_all, p, c->b_eps);
  e.n_nodes = c->n_nodes;
  e.lvl_start_host = c->hh.lvl_start;
  e.depth = c->depth;
  e.upward_done = upward_done;
  e.up_done = c->up_done;
  HIPCHK(c, launch_evaluate(c->t, e, c->stream));
  count_evaluation(c, n_req, reqs);
  return FMM_OK;
}

extern "C" fmm_status fmm_forces_batched(fmm_ctx *c, int n_req, const fmm_request *reqs,
                                         double eps, double theta, int p) {
  if (c && (p < 1 || p > c->prm.p_max || !eval_order_supported(p)))
    return fail(c, FMM_EINVAL, "order p=%d unsupported", p);
  bool evaluated = false, upward = false;
  fmm_status st = build_impl(c, n_req, reqs, eps, theta, p, &evaluated, &upward);
  if (st != FMM_OK || evaluated) return st;
  return evaluate_impl(c, n_req, reqs, p, upward);
}

static fmm_request one_request(const double *pos, const double *mass, int64_t n_total,
                               const int32_t *active, int64_t n_active, double *acc, double *pot) {
  fmm_request q = {};
  q.pos = pos;
  q.n_total = n_total;
  q.active = active;
  q.n_active = n_active;
  q.mass = mass;
  q.acc = acc;
  q.pot = pot;
  return q;
}

extern "C" fmm_status fmm_build(fmm_ctx *c, const double *pos, int64_t n_total,
                                const int32_t *active, int64_t n_active, double eps,
                                double theta) {
  fmm_request q = one_request(pos, nullptr, n_total, active, n_active, nullptr, nullptr);
  return fmm_build_batched(c, 1, &q, eps, theta);
}

extern "C" fmm_status fmm_evaluate(fmm_ctx *c, const double *pos, const double *mass,
                                   int64_t n_total, const int32_t *active, int64_t n_active, int p,
                                   double *acc, double *pot) {
  fmm_request q = one_request(pos, mass, n_total, active, n_active, acc, pot);
  return fmm_evaluate_batched(c, 1, &q, p);
}

extern "C" fmm_status fmm_forces(fmm_ctx *c, const double *pos, const double *mass,
                                 int64_t n_total, const int32_t *active, int64_t n_active,
                                 double eps, double theta, int p, double *acc, double *pot) {
  fmm_request q = one_request(pos, mass, n_total, active, n_active, acc, pot);
  return fmm_forces_batched(c, 1, &q, eps, theta, p);
}

extern "C" fmm_status fmm_forces_grad(fmm_ctx *c, const double *pos, const double *mass,
                                      int64_t n_total, const int32_t *active, int64_t n_active,
                                      double eps, double theta, int p, double *acc, double *pot,
                                      double *grad) {
  if (!c) return FMM_EINVAL;
  if (n_active > 0 && !grad) return fail(c, FMM_EINVAL, "grad is NULL");
  if (!c->gstage && !dalloc(c, &c->gstage, 6 * c->max_n))
    return fail(c, FMM_ENOMEM, "force-gradient staging");
  fmm_status st = fmm_forces(c, pos, mass, n_total, active, n_active, eps, theta, p, acc, pot);
  if (st != FMM_OK || n_active == 0) return st;
  HIPCHK(c, launch_force_gradient(c->t, c->n_nodes, (int)n_active, p, c->prm.kernel,
                                  c->prm.precision == FMM_PREC_MIXED, eps, c->gstage, grad,
                                  c->stream));
  return FMM_OK;
}

extern "C" fmm_status fmm_evaluate_dipole(fmm_ctx *c, const double *pos, const double *mass,
                                          int64_t n_total, const int32_t *active,
                                          int64_t n_active, int p, const double *vec, double *u,
                                          double *phi) {
  if (!c) return FMM_EINVAL;
  if (n_active > 0 && (!vec || !u || !phi || !mass))
    return fail(c, FMM_EINVAL, "NULL mass, vec, u or phi");
  if (c->tree_valid && c->b_reqs.size() != 1)
    return fail(c, FMM_EINVAL, "the vector-source pass needs a single-system tree");
  fmm_request q = one_request(pos, mass, n_total, active, n_active, u, phi);
  int64_t n_all = 0;
  fmm_status st = check_requests(c, 1, &q, true, &n_all);
  if (st != FMM_OK) return st;
  const fmm_request &b = c->b_reqs.empty() ? q : c->b_reqs[0];
  if (!c->tree_valid || b.pos != pos || b.active != active || b.n_active != n_active ||
      b.n_total != n_total)
    return fail(c, FMM_ESTALE, "no tree built for these particles");
  if (p < 1 || p > c->prm.p_max || !eval_order_supported(p))
    return fail(c, FMM_EINVAL, "order p=%d unsupported (1..%d)", p, std::min(c->prm.p_max, 6));
  if (n_active == 0) return FMM_OK;
  if (!c->dvec && !dalloc(c, &c->dvec, 3 * c->max_n))
    return fail(c, FMM_ENOMEM, "vector-source scratch");
  st = upload_requests(c, 1, &q, nullptr);
  if (st != FMM_OK) return st;
  EvalArgs e = {};
  set_eval_args(c, e, n_all, p, c->b_eps);
  e.n_nodes = c->n_nodes;
  e.lvl_start_host = c->hh.lvl_start;
  e.depth = c->depth;
  HIPCHK(c, launch_dipole(c->t, e, vec, c->dvec, c->stream));
  return FMM_OK;
}

extern "C" fmm_status fmm_tree_info(fmm_ctx *c, int64_t info[9]) {
  if (!c || !info) return FMM_EINVAL;
  if (!c->tree_valid) return fail(c, FMM_ESTALE, "no tree");
  const Header &h = c->hh;
  int64_t leaves = h.n_leaves;
  info[0] = c->b_n;  // active particles over all requests
  info[1] = c->n_nodes;
  info[2] = h.m2l_cursor / 2;
  info[3] = ((int64_t)h.p2p_cursor - leaves) / 2 + leaves;
  info[4] = c->depth;
  info[5] = leaves;
  info[6] = h.m2l_cursor;
  info[7] = h.p2p_cursor;
  info[8] = (int64_t)h.p2p_pairs;
  return FMM_OK;
}

template <typename T>
static hipError_t d2h(std::vector<T> &v, const T *d, int64_t n, hipStream_t s) {
  v.resize((size_t)std::max<int64_t>(n, 0));
  if (n <= 0) return hipSuccess;
  return hipMemcpyAsync(v.data(), d, sizeof(T) * n, hipMemcpyDeviceToHost, s);
}

extern "C" fmm_status fmm_export_tree(fmm_ctx *c, int64_t *perm, int32_t *level, uint64_t *prefix,
                                      int64_t *begin, int64_t *end, int32_t *is_leaf,
                                      double *centre, double *half, int64_t *m2l_pairs,
                                      int64_t *p2p_pairs, double *box) {
  if (!c) return FMM_EINVAL;
  if (!c->tree_valid) return fail(c, FMM_ESTALE, "no tree");
  if (c->b_reqs.size() != 1) return fail(c, FMM_EINVAL, "export needs a single-request tree");
  const int64_t n = c->b_n, nn = c->n_nodes;
  const DevTree &t = c->t;
  std::vector<int32_t> nbeg, nend, nlev, nnch, slot, moff, mcnt, msrc, poff, pcnt, psrc;
  std::vector<uint64_t> key;
  std::vector<double4> geo;
  Box hb;
  hipStream_t s = c->stream;
  // single request: slot == active slot
  HIPCHK(c, d2h(nbeg, t.nbeg, nn, s));
  HIPCHK(c, d2h(nend, t.nend, nn, s));
  HIPCHK(c, d2h(nlev, t.nlev, nn, s));
  HIPCHK(c, d2h(nnch, t.nnchild, nn, s));
  HIPCHK(c, d2h(geo, t.ngeo, nn, s));
  HIPCHK(c, d2h(slot, t.slot, n, s));
  HIPCHK(c, d2h(key, t.key, n, s));
  HIPCHK(c, d2h(moff, t.m2l_off, nn, s));
  HIPCHK(c, d2h(mcnt, t.m2l_cnt, nn, s));
  HIPCHK(c, d2h(poff, t.p2p_off, nn, s));
  HIPCHK(c, d2h(pcnt, t.p2p_cnt, nn, s));
  HIPCHK(c, d2h(msrc, t.m2l_src, (int64_t)c->hh.m2l_cursor, s));
  HIPCHK(c, d2h(psrc, t.p2p_src, (int64_t)c->hh.p2p_cursor, s));
  HIPCHK(c, hipMemcpyAsync(&hb, t.box, sizeof(Box), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  // canonical pre-order id: nodes sorted by (begin, level)
  std::vector<int64_t> order(nn), canon(nn);
  for (int64_t i = 0; i < nn; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    if (nbeg[a] != nbeg[b]) return nbeg[a] < nbeg[b];
    return nlev[a] < nlev[b];
  });
  for (int64_t r = 0; r < nn; ++r) canon[order[r]] = r;
  if (perm)
    for (int64_t i = 0; i < n; ++i) perm[i] = slot[i];
  for (int64_t r = 0; r < nn; ++r) {
    int64_t i = order[r];
    if (level) level[r] = nlev[i];
    if (prefix) prefix[r] = key[nbeg[i]] >> (3 * (FMM_MAXLEVEL - nlev[i]));
    if (begin) begin[r] = nbeg[i];
    if (end) end[r] = nend[i];
    if (is_leaf) is_leaf[r] = nnch[i] == 0;
    if (centre) {
      centre[3 * r] = geo[i].x;
      centre[3 * r + 1] = geo[i].y;
      centre[3 * r + 2] = geo[i].z;
    }
    if (half) half[r] = geo[i].w;
  }
  auto pairs = [&](const std::vector<int32_t> &off, const std::vector<int32_t> &cnt,
                   const std::vector<int32_t> &src, int64_t *out) {
    std::vector<std::pair<int64_t, int64_t>> v;
    for (int64_t a = 0; a < nn; ++a)
      for (int q = 0; q < cnt[a]; ++q) {
        int64_t b = src[off[a] + q];
        int64_t ca = canon[a], cb = canon[b];
        if (ca <= cb) v.emplace_back(ca, cb);
      }
    std::sort(v.begin(), v.end());
    for (size_t k = 0; k < v.size(); ++k) {
      out[2 * k] = v[k].first;
      out[2 * k + 1] = v[k].second;
    }
  };
  if (m2l_pairs) pairs(moff, mcnt, msrc, m2l_pairs);
  if (p2p_pairs) pairs(poff, pcnt, psrc, p2p_pairs);
  if (box) {
    box[0] = hb.o[0];
    box[1] = hb.o[1];
    box[2] = hb.o[2];
    box[3] = hb.L;
    box[4] = hb.s;
  }
  return FMM_OK;
}

extern "C" fmm_status fmm_invariants(fmm_ctx *c, const double *pos, const double *vel,
                                     const double *mass, const double *acc, const double *pot,
                                     int64_t n, double out[12]) {
  if (!c || !out || n < 0) return FMM_EINVAL;
  const int nblk = FMM_INV_BLOCKS;
  launch_invariants(pos, vel, mass, acc, pot, n, c->inv_part, nblk, c->stream);
  std::vector<double> part(nblk * 12);
  HIPCHK(c, hipMemcpyAsync(part.data(), c->inv_part, sizeof(double) * nblk * 12,
                           hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < 12; ++k) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[b * 12 + k];
    out[k] = s;
  }
  return FMM_OK;
}

extern "C" fmm_status fmm_profile_enable(fmm_ctx *c, int enable) {
  if (!c) return FMM_EINVAL;
  PhaseTimer &tm = c->timer;
  if (enable && !tm.ready) {
    for (int i = 0; i < PhaseTimer::CAP; ++i) {
      HIPCHK(c, hipEventCreate(&tm.a[i]));
      HIPCHK(c, hipEventCreate(&tm.b[i]));
    }
    tm.ready = true;
  }
  if (tm.on) tm.flush();
  tm.on = enable != 0;
  tm.mask = enable == 2 ? (1u << PH_M2L | 1u << PH_P2P) : ~0u;
  tm.n = 0;
  for (int k = 0; k < PH_N; ++k) {
    tm.ms[k] = 0.0;
    tm.cnt[k] = 0;
  }
  return FMM_OK;
}

extern "C" fmm_status fmm_profile_read(fmm_ctx *c, double ms[7], int64_t calls[7]) {
  if (!c || !ms || !calls) return FMM_EINVAL;
  c->timer.flush();
  for (int k = 0; k < PH_N; ++k) {
    ms[k] = c->timer.ms[k];
    calls[k] = c->timer.cnt[k];
  }
  return FMM_OK;
}
