// Request server for ensembles of independent HHS simulations (continuous
// batching).  Every request is one system advanced with the HHS integrator
// (Sec. 2.2, Algorithms 1-3) from its initial state to t_end.
//
// All device memory of resident requests comes from one arena allocated at
// creation.  A request is admitted, in arrival order, when a slot is free and
// its footprint (state + integrator scratch) fits in the arena; it is then
// resident until it finishes.  serve_step runs rounds of the batched HHS
// driver over all resident requests: in a round every request advances until
// it needs the device (a split count or a KDK half), then all pending split
// counts are read back at once, or all pending KDK halves are solved in shared
// launches.  A request that ends its top-level step begins the next one in
// the same round, and a request admitted between rounds joins the next one,
// so requests at different points of their steps (and of different depths)
// share launches instead of waiting for the slowest to end its step.  Every
// request follows exactly the operations of a run of it alone, so its result
// does not depend on what it was served with.
#include <math.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <memory>
#include <type_traits>
#include <vector>

#include "../../include/fmm355.h"
#include "context.h"
#include "hhs_driver.h"

namespace {

constexpr int64_t kAlign = 256;

int64_t align_up(int64_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// First-fit sub-allocator over one device block; free ranges are kept sorted
// by offset and merged with their neighbours on release.
struct Arena {
  char *base = nullptr;
  int64_t size = 0, used = 0;
  std::map<int64_t, int64_t> free_;  // offset -> length

  void reset(char *b, int64_t s) {
    base = b;
    size = s;
    used = 0;
    free_.clear();
    if (s > 0) free_[0] = s;
  }
  bool alloc(int64_t bytes, int64_t *off) {
    bytes = align_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const int64_t rest = it->second - bytes;
      const int64_t at = it->first + bytes;
      free_.erase(it);
      if (rest > 0) free_[at] = rest;
      used += bytes;
      return true;
    }
    return false;
  }
  void release(int64_t off, int64_t bytes) {
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
};

// Device layout of one request's state arrays ahead of its integrator
// scratch; returns the bytes, sets the pointers when base is not NULL.
int64_t state_layout(hhs_state *st, char *base, int64_t n) {
  int64_t off = 0;
  auto take = [&](auto **p, int64_t count) {
    using T = std::remove_pointer_t<std::remove_pointer_t<decltype(p)>>;
    off = align_up(off);
    if (base) *p = (T *)(base + off);
    off += count * (int64_t)sizeof(T);
  };
  hhs_state tmp;
  hhs_state *q = base ? st : &tmp;
  double *mass = nullptr;
  take(&q->pos, 3 * n);
  take(&q->vel, 3 * n);
  take(&mass, n);
  take(&q->a_old, n);
  take(&q->a_cur, n);
  take(&q->a_tot, n);
  take(&q->rung, n);
  if (base) q->mass = mass;
  return align_up(off);
}

struct Req {
  int64_t id;
  serve_request rq;
  double t_submit, t_admit;
  int64_t off, bytes;  // arena block
  hhs_state st;
  hhs_run *run;
  HhsSys *sys;  // its frame stack in the batched driver
  int slot;     // its split counter, one of [0, max_slots)
  double dt_top, dt_cur;
  bool stepping, last;  // a step of dt_cur is in progress; it ends at t_end
  int64_t steps;
};

// Host time after which serve_step returns between rounds, so that the caller
// can hand over requests that arrived meanwhile.
constexpr double kQuantum = 2e-3;

}  // namespace

struct fmm_server {
  fmm_ctx *ctx;
  hhs_params hp;
  serve_params sp;
  void *block;
  Arena arena;
  std::deque<std::unique_ptr<Req>> queue;
  std::vector<std::unique_ptr<Req>> resident;
  std::deque<serve_result> done;
  int64_t next_id, ticks;
  std::vector<int> free_slots;
  double *dmin;  // [max_slots] device minima of |a| at admission
  std::vector<double> hmin;
  std::chrono::steady_clock::time_point t0;
};

static double now_s(const fmm_server *s) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

extern "C" int64_t serve_footprint(int64_t n, int max_levels) {
  const int64_t run = hhs_run_bytes(n, max_levels);
  if (run < 0) return -1;
  return state_layout(nullptr, nullptr, n) + run;
}

extern "C" fmm_status serve_create(fmm_ctx *c, const hhs_params *hp, const serve_params *sp,
                                   fmm_server **out) {
  if (!c || !hp || !sp || !out) return FMM_EINVAL;
  if (hp->max_levels < 1 || hp->max_levels > 30 || !(hp->eta > 0) || hp->p < 1 ||
      hp->p > c->prm.p_max || !(hp->eta1 >= 0))
    return fmm_fail(c, FMM_EINVAL, "bad HHS parameters");
  if (hp->cosmo) return fmm_fail(c, FMM_EINVAL, "the server has no comoving form");
  if (sp->arena_bytes < kAlign || sp->max_slots < 1 || !(sp->dt_max > 0))
    return fmm_fail(c, FMM_EINVAL, "bad server parameters");
  fmm_server *s = new (std::nothrow) fmm_server();
  if (!s) return FMM_ENOMEM;
  s->ctx = c;
  s->hp = *hp;
  s->sp = *sp;
  s->next_id = 1;
  s->t0 = std::chrono::steady_clock::now();
  if (hipMalloc(&s->block, (size_t)sp->arena_bytes) != hipSuccess) {
    delete s;
    return fmm_fail(c, FMM_ENOMEM, "server arena of %lld bytes", (long long)sp->arena_bytes);
  }
  if (hipMalloc((void **)&s->dmin, sizeof(double) * sp->max_slots) != hipSuccess) {
    (void)hipFree(s->block);
    delete s;
    return fmm_fail(c, FMM_ENOMEM, "server minima");
  }
  s->hmin.resize(sp->max_slots);
  for (int k = sp->max_slots - 1; k >= 0; --k) s->free_slots.push_back(k);
  s->arena.reset((char *)s->block, sp->arena_bytes);
  *out = s;
  return FMM_OK;
}

static void drop_resident(fmm_server *s, Req &r) {
  hhs_run_destroy(r.run);  // waits for the stream; the run's memory is the arena's
  r.run = nullptr;
  hhs_sys_destroy(r.sys);
  r.sys = nullptr;
  s->free_slots.push_back(r.slot);
  s->arena.release(r.off, r.bytes);
}

extern "C" fmm_status serve_destroy(fmm_server *s) {
  if (!s) return FMM_EINVAL;
  (void)hipStreamSynchronize(s->ctx->stream);
  for (auto &r : s->resident) drop_resident(s, *r);
  (void)hipFree(s->dmin);
  (void)hipFree(s->block);
  delete s;
  return FMM_OK;
}

extern "C" fmm_status serve_submit(fmm_server *s, const serve_request *rq, int64_t *id) {
  if (!s || !rq) return FMM_EINVAL;
  fmm_ctx *c = s->ctx;
  if (rq->n < 1 || rq->n > c->max_n) return fmm_fail(c, FMM_EINVAL, "request size outside [1, max_n]");
  if (!rq->pos || !rq->vel || !rq->mass || !rq->pos_out || !rq->vel_out)
    return fmm_fail(c, FMM_EINVAL, "NULL request array");
  if (!(rq->t_end > 0) || !std::isfinite(rq->t_end)) return fmm_fail(c, FMM_EINVAL, "t_end");
  const int64_t need = serve_footprint(rq->n, s->hp.max_levels);
  if (need > s->sp.arena_bytes)
    return fmm_fail(c, FMM_ENOMEM, "request needs %lld bytes, the arena holds %lld",
                    (long long)need, (long long)s->sp.arena_bytes);
  auto r = std::make_unique<Req>();  // value-initialised: zero counters, NULL run
  r->id = s->next_id++;
  r->rq = *rq;
  r->t_submit = now_s(s);
  r->bytes = need;
  if (id) *id = r->id;
  s->queue.push_back(std::move(r));
  return FMM_OK;
}

// Admit queued requests in arrival order while a slot and arena space are
// free; upload their state, run the initial force solve of all of them
// together and fix each one's top-level step from it.
static fmm_status admit(fmm_server *s) {
  fmm_ctx *c = s->ctx;
  std::vector<Req *> fresh;
  while (!s->queue.empty() && (int)s->resident.size() < s->sp.max_slots) {
    Req &r = *s->queue.front();
    int64_t off;
    if (!s->arena.alloc(r.bytes, &off)) break;
    r.off = off;
    char *base = s->arena.base + off;
    const int64_t n = r.rq.n;
    const int64_t sb = state_layout(&r.st, base, n);
    r.st.n = n;
    r.st.t = 0.0;
    fmm_status e = hhs_run_create_at(c, n, s->hp.max_levels, base + sb, &r.run);
    if (e == FMM_OK) {
      // a slot is free: fewer than max_slots requests are resident
      r.slot = s->free_slots.back();
      r.sys = hhs_sys_create(r.run, &r.st, r.slot);
      if (!r.sys) e = fmm_fail(c, FMM_ENOMEM, "request driver state");
    }
    if (e == FMM_OK &&
        (hipMemcpyAsync(r.st.pos, r.rq.pos, 24 * n, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
         hipMemcpyAsync(r.st.vel, r.rq.vel, 24 * n, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
         hipMemcpyAsync((double *)r.st.mass, r.rq.mass, 8 * n, hipMemcpyHostToDevice, c->stream) !=
             hipSuccess ||
         hipMemsetAsync(r.st.rung, 0, 4 * n, c->stream) != hipSuccess))
      e = fmm_fail(c, FMM_EDEVICE, "request upload failed");
    if (e != FMM_OK) {
      if (r.run) hhs_run_destroy(r.run);
      r.run = nullptr;
      hhs_sys_destroy(r.sys);
      r.sys = nullptr;
      s->arena.release(off, r.bytes);
      return e;
    }
    s->free_slots.pop_back();
    r.t_admit = now_s(s);
    s->resident.push_back(std::move(s->queue.front()));
    s->queue.pop_front();
    fresh.push_back(s->resident.back().get());
  }
  if (fresh.empty()) return FMM_OK;
  std::vector<hhs_run *> runs;
  std::vector<hhs_state *> sts;
  for (Req *r : fresh) {
    runs.push_back(r->run);
    sts.push_back(&r->st);
  }
  fmm_status e = hhs_init_batched(c, (int)fresh.size(), runs.data(), sts.data(), &s->hp);
  if (e != FMM_OK) return e;
  for (size_t k = 0; k < fresh.size(); ++k) hhs_run_launch_min_amag(fresh[k]->run, &fresh[k]->st, s->dmin + k);
  if (hipMemcpyAsync(s->hmin.data(), s->dmin, sizeof(double) * fresh.size(), hipMemcpyDeviceToHost,
                     c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return fmm_fail(c, FMM_EDEVICE, "admission readback failed");
  // top-level step: the largest particle step sqrt(eta eps / |a|) rounded
  // down to a power of two, capped at dt_max
  for (size_t k = 0; k < fresh.size(); ++k) {
    const double amin = s->hmin[k];
    double dt = s->sp.dt_max;
    if (amin > 0 && std::isfinite(amin)) {
      int ex;
      (void)frexp(sqrt(s->hp.eta * s->hp.eps / amin), &ex);
      dt = std::min(dt, ldexp(1.0, ex - 1));
    }
    fresh[k]->dt_top = dt;
  }
  return FMM_OK;
}

// Retires the finished requests of the resident list (outputs downloaded,
// results recorded, memory and slot freed), keeping the others in order.
static fmm_status retire(fmm_server *s) {
  fmm_ctx *c = s->ctx;
  for (auto &rp : s->resident) {
    Req &r = *rp;
    if (r.stepping || !r.last) continue;
    if (hipMemcpyAsync(r.rq.pos_out, r.st.pos, 24 * r.rq.n, hipMemcpyDeviceToHost, c->stream) !=
            hipSuccess ||
        hipMemcpyAsync(r.rq.vel_out, r.st.vel, 24 * r.rq.n, hipMemcpyDeviceToHost, c->stream) !=
            hipSuccess)
      return fmm_fail(c, FMM_EDEVICE, "result download failed");
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess)
    return fmm_fail(c, FMM_EDEVICE, "result download failed");
  const double t = now_s(s);
  std::vector<std::unique_ptr<Req>> keep;
  for (auto &rp : s->resident) {
    if (rp->stepping || !rp->last) {
      keep.push_back(std::move(rp));
      continue;
    }
    serve_result res;
    res.id = rp->id;
    res.n = rp->rq.n;
    res.steps = rp->steps;
    hhs_sys_counts(rp->sys, &res.force_calls, &res.force_particles);
    res.dt_top = rp->dt_top;
    res.t_end = rp->st.t;
    res.t_submit = rp->t_submit;
    res.t_admit = rp->t_admit;
    res.t_done = t;
    s->done.push_back(res);
    drop_resident(s, *rp);
  }
  s->resident.swap(keep);
  return FMM_OK;
}

extern "C" fmm_status serve_step(fmm_server *s, int *n_resident, int *n_queued) {
  if (!s) return FMM_EINVAL;
  fmm_ctx *c = s->ctx;
  const auto t_start = std::chrono::steady_clock::now();
  std::vector<HhsSys *> ps;
  for (;;) {
    fmm_status e = admit(s);
    if (e != FMM_OK) return e;
    if (s->resident.empty()) break;
    ps.clear();
    for (auto &r : s->resident) ps.push_back(r->sys);
    e = hhs_sys_advance(c, ps.data(), (int)ps.size(), &s->hp);
    if (e != FMM_OK) return e;
    // a request whose step ended is retired at t_end, else it begins its
    // next step (as does a request just admitted) and advances to its first
    // device wait, so that it joins this round
    bool restarted = false, finished = false;
    for (auto &rp : s->resident) {
      Req &r = *rp;
      if (!hhs_sys_idle(r.sys)) continue;
      if (r.stepping) {
        r.stepping = false;
        r.st.t += r.dt_cur;
        r.steps++;
        if (r.last) {
          finished = true;
          continue;
        }
      }
      const double left = r.rq.t_end - r.st.t;
      r.last = r.dt_top >= left;
      r.dt_cur = r.last ? left : r.dt_top;
      hhs_sys_begin(r.sys, r.dt_cur);
      r.stepping = true;
      restarted = true;
    }
    if (restarted) {
      e = hhs_sys_advance(c, ps.data(), (int)ps.size(), &s->hp);
      if (e != FMM_OK) return e;
    }
    if (finished) {
      e = retire(s);
      if (e != FMM_OK) return e;
      ps.clear();
      for (auto &r : s->resident) ps.push_back(r->sys);
    }
    bool served = false;
    int64_t kicks = 0;
    if (!ps.empty()) {
      e = hhs_sys_serve(c, ps.data(), (int)ps.size(), &s->hp, &kicks, &served);
      if (e != FMM_OK) return e;
    }
    ++s->ticks;
    const double spent =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    if (finished || !served || spent >= kQuantum) break;
  }
  if (n_resident) *n_resident = (int)s->resident.size();
  if (n_queued) *n_queued = (int)s->queue.size();
  return FMM_OK;
}

extern "C" fmm_status serve_poll(fmm_server *s, serve_result *out, int max_out, int *n_out) {
  if (!s || !n_out || (max_out > 0 && !out)) return FMM_EINVAL;
  int k = 0;
  while (k < max_out && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  *n_out = k;
  return FMM_OK;
}

extern "C" fmm_status serve_cancel(fmm_server *s, int64_t id) {
  if (!s) return FMM_EINVAL;
  for (auto it = s->queue.begin(); it != s->queue.end(); ++it)
    if ((*it)->id == id) {
      s->queue.erase(it);
      return FMM_OK;
    }
  for (auto it = s->resident.begin(); it != s->resident.end(); ++it)
    if ((*it)->id == id) {
      drop_resident(s, **it);
      s->resident.erase(it);
      return FMM_OK;
    }
  return fmm_fail(s->ctx, FMM_EINVAL, "no queued or resident request %lld", (long long)id);
}

extern "C" fmm_status serve_info(const fmm_server *s, int64_t info[6]) {
  if (!s || !info) return FMM_EINVAL;
  info[0] = (int64_t)s->resident.size();
  info[1] = (int64_t)s->queue.size();
  info[2] = (int64_t)s->done.size();
  info[3] = s->arena.used;
  info[4] = s->arena.size;
  info[5] = s->ticks;
  return FMM_OK;
}
