// HHS integrator driver (Sec. 2.2, Algorithms 1-3) for one or many
// independent systems.
//
// Each system's EVOLVE_HOLD recursion is an explicit frame stack.  A system
// runs on the host until it needs either the size of a slow/fast split (a
// device count) or a KDK half: the force solve(s) of Algorithm 2 at one set of
// positions -- one tree over the system, then up to two evaluations
// (kickS2F with the fast masses zeroed, kickFS2S with all masses) each followed
// by its kick.  The driver then serves every waiting system at once: one
// readback for all pending splits, or one batched tree build and two batched
// evaluation slots for all systems waiting on a half (a system with nothing to
// evaluate in a slot is skipped).  Kicks of one half act on disjoint particle
// sets and the evaluations do not read velocities, so every system follows
// exactly the sequence it would follow alone.
#include <math.h>

#include <algorithm>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/fmm355.h"
#include "common.h"
#include "context.h"
#include "hhs_driver.h"
#include "hhs_kernels.h"

// cosmo.hip: H(a) of a comoving-factor table's cosmology
double cosmo_hubble(const fmm_cosmo *c, double a);

struct hhs_run {
  fmm_ctx *ctx;
  int64_t n;
  int levels;
  void *owned;  // device block of the run, or NULL when carved from caller memory
  int32_t *all_idx;
  uint32_t *flag, *scan_part;
  uint8_t *sinks;  // sink flags of one evaluation over the joint set
  std::vector<int32_t *> slow, slow_pos, fast, fast_pos;  // per rung
  std::vector<uint8_t *> fflag, sflag;  // per rung: fast / slow flags by joint-set position
  double *mmask, *acc, *pot;
};

// Lays the run's arrays out in one block (256-byte aligned pieces); returns
// the block size, and sets the pointers when base is not NULL.
static int64_t run_layout(hhs_run *r, char *base, int64_t n, int levels) {
  int64_t off = 0;
  auto take = [&](auto **p, int64_t count) {
    using T = std::remove_pointer_t<std::remove_pointer_t<decltype(p)>>;
    off = (off + 255) & ~(int64_t)255;
    if (base) *p = (T *)(base + off);
    off += std::max<int64_t>(count, 1) * (int64_t)sizeof(T);
  };
  hhs_run tmp;
  hhs_run *q = base ? r : &tmp;
  q->slow.resize(levels);
  q->slow_pos.resize(levels);
  q->fast.resize(levels);
  q->fast_pos.resize(levels);
  q->fflag.resize(levels);
  q->sflag.resize(levels);
  take(&q->all_idx, n);
  take(&q->flag, n);
  take(&q->sinks, n);
  take(&q->scan_part, n / 1024 + 64);
  take(&q->mmask, n);
  take(&q->acc, 3 * n);
  take(&q->pot, n);
  for (int l = 0; l < levels; ++l) {
    take(&q->slow[l], n);
    take(&q->slow_pos[l], n);
    take(&q->fast[l], n);
    take(&q->fast_pos[l], n);
    take(&q->fflag[l], n);
    take(&q->sflag[l], n);
  }
  return (off + 255) & ~(int64_t)255;
}

extern "C" int64_t hhs_run_bytes(int64_t n, int max_levels) {
  if (n < 1 || max_levels < 1 || max_levels > 30) return -1;
  return run_layout(nullptr, nullptr, n, max_levels + 1);
}

fmm_status hhs_run_create_at(fmm_ctx *c, int64_t n, int max_levels, void *mem, hhs_run **out) {
  if (!c || !out || n < 1 || n > INT32_MAX || max_levels < 1 || max_levels > 30) return FMM_EINVAL;
  hhs_run *r = new (std::nothrow) hhs_run();
  if (!r) return FMM_ENOMEM;
  r->ctx = c;
  r->n = n;
  r->levels = max_levels + 1;
  if (!mem) {
    if (hipMalloc(&r->owned, (size_t)run_layout(nullptr, nullptr, n, r->levels)) != hipSuccess) {
      delete r;
      return FMM_ENOMEM;
    }
    mem = r->owned;
  }
  run_layout(r, (char *)mem, n, r->levels);
  hhs_launch_iota(r->all_idx, (int)n, c->stream);
  *out = r;
  return FMM_OK;
}

extern "C" fmm_status hhs_run_create(fmm_ctx *c, int64_t n, int max_levels, hhs_run **out) {
  return hhs_run_create_at(c, n, max_levels, nullptr, out);
}

extern "C" fmm_status hhs_run_destroy(hhs_run *r) {
  if (!r) return FMM_EINVAL;
  if (r->ctx) (void)hipStreamSynchronize(r->ctx->stream);
  if (r->owned) (void)hipFree(r->owned);
  delete r;
  return FMM_OK;
}

void hhs_run_launch_min_amag(hhs_run *r, const hhs_state *st, double *out) {
  hhs_launch_min_sum(st->a_old, st->a_cur, st->n, r->pot, out, r->ctx->stream);
}

// One level of a system's EVOLVE_HOLD recursion.
struct HhsFrame {
  int k;
  const int32_t *sys;
  int n_sys;
  double dt;
  bool calc;
  int pc;
  int n_fast, n_slow;
  double t0;  // start of the frame's step (ln a in the comoving form)
};

enum HhsSysState { S_RUN, S_WAIT_SPLIT, S_WAIT_HALF, S_DONE };

// One system of a batched run; its frame stack persists between rounds.
struct HhsSys {
  hhs_run *run;
  hhs_state *st;
  int slot;  // its split counter (c->split_cnt[slot]), fixed for its life
  double dt_top;
  std::vector<HhsFrame> stack;
  HhsSysState state;
  int half;
  int64_t kicks, parts;  // force evaluations of this system, and their active particles
  bool range_err;        // a comoving factor fell outside the cosmology table
};

namespace {

using Frame = HhsFrame;
using Sys = HhsSys;

// Comoving form (Sec. 3.5): the factor that replaces the length of a kick
// (integral of dt/a) or a drift (integral of dt/a^2) over [x0, x0 + dx] in
// ln a; the plain length dx otherwise.
bool step_factor(const hhs_params *hp, double x0, double dx, bool kick, double *out) {
  if (!hp->cosmo) {
    *out = dx;
    return true;
  }
  double d, k;
  if (fmm_cosmo_factors(hp->cosmo, exp(x0), exp(x0 + dx), &d, &k) != FMM_OK) return false;
  *out = kick ? k : d;
  return true;
}

// One kick of Algorithm 3 inside a KDK half: which set is kicked, with which
// masses, and which |a| slot a second kick refreshes.
struct Kick {
  bool s2f;     // kickS2F (fast sinks, fast masses zeroed) or kickFS2S
  bool second;  // second kick of the KDK
};

int kicks_of_half(const Frame &f, int half, Kick out[2]) {
  const bool s2f = f.n_fast > 0 && f.n_slow > 0;
  int n = 0;
  if (half == 0) {
    if (s2f) out[n++] = {true, false};
    if (f.n_slow) out[n++] = {false, false};
  } else {
    if (f.n_slow) out[n++] = {false, true};
    if (s2f) out[n++] = {true, true};
  }
  return n;
}

// Runs system S until it waits on the device or finishes; false when the
// rung recursion would go deeper than the scratch holds.  The rung
// assignment + split and the drift it reaches are appended to splits and
// drifts, which the caller launches (batched over systems) before anything
// else is queued for S.
struct SplitReq {
  HhsSplitItem it;
  hhs_run *run;  // its scan scratch, for the multi-workgroup split
};

bool advance(fmm_ctx *c, Sys &S, const hhs_params *hp, std::vector<SplitReq> &splits,
             std::vector<HhsDriftItem> &drifts) {
  const int slot = S.slot;
  hhs_run *r = S.run;
  hhs_state *st = S.st;
  while (S.state == S_RUN) {
    if (S.stack.empty()) {
      S.state = S_DONE;
      return true;
    }
    Frame &f = S.stack.back();
    const int k = f.k;
    if (k >= r->levels) return false;
    switch (f.pc) {
      case 0: {  // (re)assign rungs, split into slow {rung <= k} and fast {rung > k}
        HhsSplitItem it{};
        it.sys = f.sys;
        it.n_sys = f.n_sys;
        it.rung = st->rung;
        it.k = k;
        it.slow = r->slow[k];
        it.slow_pos = r->slow_pos[k];
        it.fast = r->fast[k];
        it.fast_pos = r->fast_pos[k];
        it.count = c->split_cnt + slot;
        it.fflag = r->fflag[k];
        it.sflag = r->sflag[k];
        it.do_rungs = f.calc && !hp->freeze_rungs;
        if (it.do_rungs) {
          // comoving form: a rung's step in ln a is compared in physical
          // time, d(ln a) / H at the start of the subsystem's step
          double h2 = 1.0;
          if (hp->cosmo) {
            const double H = cosmo_hubble(hp->cosmo, exp(f.t0));
            h2 = H * H;
          }
          it.a_old = st->a_old;
          it.a_cur = st->a_cur;
          it.a_tot = hp->eta1 > 0 ? st->a_tot : nullptr;
          it.dt_top = S.dt_top;
          it.eta_eps = (hp->eta * hp->eps) * h2;
          it.eta1_eps = (hp->eta1 * hp->eps) * h2;
          it.max_levels = hp->max_levels;
        }
        splits.push_back(SplitReq{it, r});
        f.pc = 1;
        S.state = S_WAIT_SPLIT;
        return true;
      }
      case 1: {  // first half of the fast system's evolution
        f.pc = 2;
        if (f.n_fast > 0) {
          Frame ch{k + 1, r->fast[k], f.n_fast, 0.5 * f.dt, false, 0, 0, 0, f.t0};
          S.stack.push_back(ch);
        }
        break;
      }
      case 2:  // KDK, first half: kicks at the current positions
        f.pc = 3;
        if ((f.n_fast > 0 && f.n_slow > 0) || f.n_slow > 0) {
          S.half = 0;
          S.state = S_WAIT_HALF;
          return true;
        }
        break;
      case 3: {  // drift the slow system, second half of the KDK
        double fd;
        if (!step_factor(hp, f.t0, f.dt, false, &fd)) {
          S.range_err = true;
          return false;
        }
        if (f.n_slow > 0)
          drifts.push_back(HhsDriftItem{r->slow[k], st->vel, st->pos, st->n, fd, f.n_slow});
        f.pc = 4;
        if ((f.n_fast > 0 && f.n_slow > 0) || f.n_slow > 0) {
          S.half = 1;
          S.state = S_WAIT_HALF;
          return true;
        }
        break;
      }
      case 4: {  // second half of the fast system's evolution, rungs recomputed
        f.pc = 5;
        if (f.n_fast > 0) {
          Frame ch{k + 1, r->fast[k], f.n_fast, 0.5 * f.dt, true, 0, 0, 0, f.t0 + 0.5 * f.dt};
          S.stack.push_back(ch);
        }
        break;
      }
      default:
        S.stack.pop_back();
        break;
    }
  }
  return true;
}

}  // namespace

// The KDK halves of W waiting systems: their trees in one batched build, then
// the kicks of the half in two batched evaluation slots (a system with no kick
// in a slot is skipped there), each followed by its systems' kicks; the build
// and the first slot's evaluation are one fmm_forces_batched call.  Each
// evaluation takes the kicked set as its sinks (P2P skips leaves without one);
// the second kickFS2S of a top-level KDK evaluates the whole system when the
// bound of Eq. 9 needs |a|_tot.
static fmm_status serve_half(fmm_ctx *c, HhsSys *const *sys, const int *grp, int W,
                             const hhs_params *hp, int64_t *kicks) {
  std::vector<fmm_request> q(W);
  std::vector<Kick> kk(2 * W, Kick{false, false});
  std::vector<int> nk(W);
  for (int w = 0; w < W; ++w) {
    Sys &S = *sys[grp[w]];
    const Frame &f = S.stack.back();
    q[w] = fmm_request{S.st->pos, S.st->n, f.sys, f.n_sys, nullptr, S.run->acc, S.run->pot};
    nk[w] = kicks_of_half(f, S.half, &kk[2 * w]);
  }
  fmm_status e;
  for (int slot = 0; slot < 2; ++slot) {
    bool any = false;
    std::vector<HhsMaskItem> masks;
    for (int w = 0; w < W; ++w) {
      Sys &S = *sys[grp[w]];
      const Frame &f = S.stack.back();
      q[w].mass = nullptr;
      if (slot >= nk[w]) continue;
      any = true;
      const Kick &K = kk[2 * w + slot];
      if (K.s2f) {
        masks.push_back(HhsMaskItem{f.sys, S.run->fflag[f.k], S.st->mass, S.run->mmask, f.n_sys});
        q[w].mass = S.run->mmask;
      } else {
        q[w].mass = S.st->mass;
      }
      const int n_set = K.s2f ? f.n_fast : f.n_slow;
      const bool all = n_set == f.n_sys ||
                       (!K.s2f && K.second && f.k == 0 && hp->eta1 > 0 && S.st->a_tot);
      // the kicked set's flags by joint-set position, written by the split
      q[w].sinks = all ? nullptr : K.s2f ? S.run->fflag[f.k] : S.run->sflag[f.k];
    }
    hhs_launch_masked_masses(masks.data(), (int)masks.size(), c->stream);
    if (slot == 0) {
      // the first slot's masses and sinks are known before the tree: one call
      // builds and evaluates (upward pass beside the walk, the evaluation
      // queued behind the walk without a host wait between them)
      e = any ? fmm_forces_batched(c, W, q.data(), hp->eps, hp->theta, hp->p)
              : fmm_build_batched(c, W, q.data(), hp->eps, hp->theta);
      if (e != FMM_OK) return e;
      if (!any) continue;
    } else {
      if (!any) continue;
      e = fmm_evaluate_batched(c, W, q.data(), hp->p);
      if (e != FMM_OK) return e;
    }
    std::vector<HhsKickItem> kick_items;
    std::vector<int> norms;  // systems whose solve also gives |a|_tot
    for (int w = 0; w < W; ++w) {
      if (slot >= nk[w]) continue;
      Sys &S = *sys[grp[w]];
      const Frame &f = S.stack.back();
      const Kick &K = kk[2 * w + slot];
      const int k = f.k;
      // first kicks cover [t0, t0 + dt/2], second ones [t0 + dt/2, t0 + dt]
      double fk;
      if (!step_factor(hp, S.half ? f.t0 + 0.5 * f.dt : f.t0, 0.5 * f.dt, true, &fk))
        return fmm_fail(c, FMM_EINVAL, "scale factor outside the cosmology table");
      if (K.s2f)
        kick_items.push_back(HhsKickItem{S.run->fast[k], S.run->fast_pos[k], S.run->acc,
                                         S.st->vel, K.second ? S.st->a_old : nullptr, f.n_sys,
                                         S.st->n, fk, f.n_fast});
      else
        kick_items.push_back(HhsKickItem{S.run->slow[k], S.run->slow_pos[k], S.run->acc,
                                         S.st->vel, K.second ? S.st->a_cur : nullptr, f.n_sys,
                                         S.st->n, fk, f.n_slow});
      // Eq. 9: the second kickFS2S of a top-level KDK sees every particle as a
      // sink, so its solve gives |a|_tot for the whole system
      if (!K.s2f && K.second && k == 0 && hp->eta1 > 0 && S.st->a_tot) norms.push_back(w);
      ++*kicks;
      ++S.kicks;
      S.parts += f.n_sys;
    }
    // the slot's kicks (and |a|_tot) read acc before the next slot rewrites it
    hhs_launch_kicks(kick_items.data(), (int)kick_items.size(), c->stream);
    for (int w : norms) {
      Sys &S = *sys[grp[w]];
      const Frame &f = S.stack.back();
      hhs_launch_norm_at(f.sys, f.n_sys, S.run->acc, S.st->a_tot, c->stream);
    }
  }
  return FMM_OK;
}

static fmm_status ensure_split_slots(fmm_ctx *c, int n) {
  if (n <= c->cap_split) return FMM_OK;
  if (c->split_cnt) fmm_dfree(c, c->split_cnt);
  c->split_cnt = nullptr;
  const int cap = std::max(n, 2 * c->cap_split);
  if (c->pin_split) (void)hipHostFree(c->pin_split);
  c->pin_split = nullptr;
  c->cap_split = 0;
  if (!fmm_dalloc(c, &c->split_cnt, cap)) return fmm_fail(c, FMM_ENOMEM, "split counters");
  if (hipHostMalloc((void **)&c->pin_split, sizeof(int32_t) * cap) != hipSuccess) {
    c->pin_split = nullptr;
    return fmm_fail(c, FMM_ENOMEM, "split readback buffer");
  }
  c->cap_split = cap;
  return FMM_OK;
}

static fmm_status check_system(fmm_ctx *c, hhs_run *r, hhs_state *st, const hhs_params *hp) {
  if (!r || !st) return fmm_fail(c, FMM_EINVAL, "NULL system");
  if (st->n < 1 || st->n > r->n) return fmm_fail(c, FMM_EINVAL, "state larger than its scratch");
  if (!st->pos || !st->vel || !st->mass || !st->a_old || !st->a_cur || !st->rung)
    return fmm_fail(c, FMM_EINVAL, "NULL state array");
  if (hp->max_levels + 1 > r->levels) return fmm_fail(c, FMM_EINVAL, "scratch has too few rungs");
  if (hp->eta1 > 0 && !st->a_tot)
    return fmm_fail(c, FMM_EINVAL, "eta1 > 0 needs the a_tot array");
  return FMM_OK;
}

static fmm_status check_distinct(fmm_ctx *c, int n_sys, hhs_run *const *runs,
                                 hhs_state *const *states) {
  std::vector<const void *> v;
  for (int i = 0; i < n_sys; ++i) {
    v.push_back(runs[i]);
    if (states[i]) v.push_back(states[i]->pos);
  }
  std::sort(v.begin(), v.end());
  if (std::adjacent_find(v.begin(), v.end()) != v.end())
    return fmm_fail(c, FMM_EINVAL, "systems share a run or a state");
  return FMM_OK;
}

static fmm_status check_params(fmm_ctx *c, const hhs_params *hp) {
  if (!c || !hp) return FMM_EINVAL;
  if (hp->max_levels < 1 || hp->max_levels > 30 || !(hp->eta > 0) || hp->p < 1 ||
      hp->p > c->prm.p_max || !(hp->eta1 >= 0))
    return fmm_fail(c, FMM_EINVAL, "bad HHS parameters");
  return FMM_OK;
}

extern "C" fmm_status hhs_init_batched(fmm_ctx *c, int n_sys, hhs_run *const *runs,
                                       hhs_state *const *states, const hhs_params *hp) {
  fmm_status e = check_params(c, hp);
  if (e != FMM_OK) return e;
  if (n_sys < 1 || !runs || !states) return fmm_fail(c, FMM_EINVAL, "no systems");
  e = check_distinct(c, n_sys, runs, states);
  if (e != FMM_OK) return e;
  std::vector<fmm_request> q(n_sys);
  for (int i = 0; i < n_sys; ++i) {
    e = check_system(c, runs[i], states[i], hp);
    if (e != FMM_OK) return e;
    hhs_state *st = states[i];
    q[i] = fmm_request{st->pos, st->n, nullptr, st->n, st->mass, runs[i]->acc, runs[i]->pot};
  }
  for (int g0 = 0; g0 < n_sys;) {  // groups that fit the context
    int g1 = g0;
    int64_t tot = 0;
    while (g1 < n_sys && (g1 == g0 || tot + q[g1].n_active <= c->max_n)) tot += q[g1++].n_active;
    e = fmm_forces_batched(c, g1 - g0, q.data() + g0, hp->eps, hp->theta, hp->p);
    if (e != FMM_OK) return e;
    g0 = g1;
  }
  for (int i = 0; i < n_sys; ++i) {
    hhs_launch_amag(runs[i]->acc, states[i]->n, states[i]->a_cur, states[i]->a_old, c->stream);
    if (states[i]->a_tot)
      hhs_launch_norm_at(runs[i]->all_idx, (int)states[i]->n, runs[i]->acc, states[i]->a_tot,
                         c->stream);
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess)
    return fmm_fail(c, FMM_EDEVICE, "hhs_init synchronisation failed");
  return FMM_OK;
}

HhsSys *hhs_sys_create(hhs_run *run, hhs_state *st, int slot) {
  HhsSys *S = new (std::nothrow) HhsSys();
  if (!S) return nullptr;
  S->run = run;
  S->st = st;
  S->slot = slot;
  S->state = S_DONE;
  S->half = 0;
  S->kicks = S->parts = 0;
  S->range_err = false;
  return S;
}

void hhs_sys_destroy(HhsSys *S) { delete S; }

void hhs_sys_begin(HhsSys *S, double dt_top) {
  S->dt_top = dt_top;
  S->state = S_RUN;
  S->half = 0;
  S->range_err = false;
  S->stack.clear();
  S->stack.push_back(Frame{0, S->run->all_idx, (int)S->st->n, dt_top, true, 0, 0, 0, S->st->t});
}

bool hhs_sys_idle(const HhsSys *S) { return S->state == S_DONE; }

void hhs_sys_counts(const HhsSys *S, int64_t *kicks, int64_t *parts) {
  *kicks = S->kicks;
  *parts = S->parts;
}

fmm_status hhs_sys_advance(fmm_ctx *c, HhsSys *const *sys, int n_sys, const hhs_params *hp) {
  int ns = 0;
  for (int i = 0; i < n_sys; ++i) ns = std::max(ns, sys[i]->slot + 1);
  fmm_status e = ensure_split_slots(c, ns);
  if (e != FMM_OK) return e;
  std::vector<SplitReq> splits;
  std::vector<HhsSplitItem> small, big;
  std::vector<uint32_t *> big_flag, big_part;
  std::vector<HhsDriftItem> drifts;
  for (int i = 0; i < n_sys; ++i)
    if (sys[i]->state == S_RUN && !advance(c, *sys[i], hp, splits, drifts))
      return fmm_fail(c, FMM_EINVAL,
                      sys[i]->range_err ? "system %d: scale factor outside the cosmology table"
                                        : "system %d: rung recursion deeper than max_levels",
                      i);
  // a system reaches at most one drift or split per round, and they touch
  // different arrays: the drifts first, then the splits (one workgroup per
  // joint set up to HHS_SPLIT_MAX_N, the multi-workgroup kernels beyond)
  hhs_launch_drifts(drifts.data(), (int)drifts.size(), c->stream);
  for (const SplitReq &q : splits) {
    const HhsSplitItem &it = q.it;
    if (it.n_sys <= HHS_SPLIT_MAX_N) {
      small.push_back(it);
      continue;
    }
    big.push_back(it);
    big_flag.push_back(q.run->flag);
    big_part.push_back(q.run->scan_part);
  }
  hhs_launch_splits(small.data(), (int)small.size(), c->stream);
  hhs_launch_big_splits(big.data(), big_flag.data(), big_part.data(), (int)big.size(), c->stream);
  return FMM_OK;
}

fmm_status hhs_sys_serve(fmm_ctx *c, HhsSys *const *sys, int n_sys, const hhs_params *hp,
                         int64_t *kicks, bool *served) {
  *served = false;
  std::vector<int> wait;
  int ns = 0;
  for (int i = 0; i < n_sys; ++i)
    if (sys[i]->state == S_WAIT_SPLIT) {
      wait.push_back(i);
      ns = std::max(ns, sys[i]->slot + 1);
    }
  if (!wait.empty()) {  // one readback for every pending split
    if (ns > c->cap_split) return fmm_fail(c, FMM_EINVAL, "split slot beyond the counters");
    if (hipMemcpyAsync(c->pin_split, c->split_cnt, sizeof(int32_t) * ns,
                       hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
      return fmm_fail(c, FMM_EDEVICE, "split readback failed");
    for (int i : wait) {
      Frame &f = sys[i]->stack.back();
      f.n_fast = c->pin_split[sys[i]->slot];
      f.n_slow = f.n_sys - f.n_fast;
      sys[i]->state = S_RUN;
    }
    *served = true;
    return FMM_OK;
  }
  for (int i = 0; i < n_sys; ++i)
    if (sys[i]->state == S_WAIT_HALF) wait.push_back(i);
  if (wait.empty()) return FMM_OK;
  // systems waiting on a KDK half, packed greedily into groups that fit the
  // context; one batched build and two evaluation slots per group
  size_t g0 = 0;
  while (g0 < wait.size()) {
    size_t g1 = g0;
    int64_t tot = 0;
    while (g1 < wait.size()) {
      const int64_t m = sys[wait[g1]]->stack.back().n_sys;
      if (g1 > g0 && tot + m > c->max_n) break;
      tot += m;
      ++g1;
    }
    fmm_status e = serve_half(c, sys, wait.data() + g0, (int)(g1 - g0), hp, kicks);
    if (e != FMM_OK) return e;
    g0 = g1;
  }
  for (int i : wait) sys[i]->state = S_RUN;
  *served = true;
  return FMM_OK;
}

fmm_status hhs_step_batched_ex(fmm_ctx *c, int n_sys, hhs_run *const *runs,
                               hhs_state *const *states, const hhs_params *hp,
                               const double *dt_top, int64_t stats[3], int64_t *sys_stats) {
  fmm_status e = check_params(c, hp);
  if (e != FMM_OK) return e;
  if (n_sys < 1 || !runs || !states || !dt_top) return fmm_fail(c, FMM_EINVAL, "no systems");
  e = check_distinct(c, n_sys, runs, states);
  if (e != FMM_OK) return e;
  std::vector<HhsSys> sys(n_sys);
  std::vector<HhsSys *> ps(n_sys);
  for (int i = 0; i < n_sys; ++i) {
    e = check_system(c, runs[i], states[i], hp);
    if (e != FMM_OK) return e;
    if (!std::isfinite(dt_top[i]) || dt_top[i] == 0.0)
      return fmm_fail(c, FMM_EINVAL, "dt_top of system %d", i);
    Sys &S = sys[i];
    S.run = runs[i];
    S.st = states[i];
    S.slot = i;
    S.kicks = S.parts = 0;
    hhs_sys_begin(&S, dt_top[i]);
    ps[i] = &S;
  }
  const int64_t c0 = c->stat_parts, b0 = c->stat_builds;
  int64_t kicks = 0;
  // rounds: every running system advances until it waits on the device or
  // ends its step, then either all pending splits or all pending KDK halves
  // are served; the step ends when nothing waits
  for (;;) {
    e = hhs_sys_advance(c, ps.data(), n_sys, hp);
    if (e != FMM_OK) return e;
    bool served;
    e = hhs_sys_serve(c, ps.data(), n_sys, hp, &kicks, &served);
    if (e != FMM_OK) return e;
    if (!served) break;
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess)
    return fmm_fail(c, FMM_EDEVICE, "hhs_step synchronisation failed");
  for (int i = 0; i < n_sys; ++i) states[i]->t += dt_top[i];
  if (stats) {
    stats[0] = kicks;
    stats[1] = c->stat_parts - c0;
    stats[2] = c->stat_builds - b0;
  }
  if (sys_stats)
    for (int i = 0; i < n_sys; ++i) {
      sys_stats[2 * i] = sys[i].kicks;
      sys_stats[2 * i + 1] = sys[i].parts;
    }
  c->tree_valid = false;
  return FMM_OK;
}

extern "C" fmm_status hhs_step_batched(fmm_ctx *c, int n_sys, hhs_run *const *runs,
                                       hhs_state *const *states, const hhs_params *hp,
                                       const double *dt_top, int64_t stats[3]) {
  return hhs_step_batched_ex(c, n_sys, runs, states, hp, dt_top, stats, nullptr);
}

static fmm_status own_run(fmm_ctx *c, hhs_state *st, const hhs_params *hp) {
  hhs_run *r = c->own_run;
  if (r && r->n >= st->n && r->levels >= hp->max_levels + 1) return FMM_OK;
  if (r) hhs_run_destroy(r);
  c->own_run = nullptr;
  return hhs_run_create(c, c->max_n, std::max(hp->max_levels, 16), &c->own_run);
}

extern "C" fmm_status hhs_init(fmm_ctx *c, hhs_state *st, const hhs_params *hp) {
  fmm_status e = check_params(c, hp);
  if (e != FMM_OK) return e;
  if (!st) return FMM_EINVAL;
  if (st->n < 1 || st->n > c->max_n) return fmm_fail(c, FMM_EINVAL, "state size outside [1, max_n]");
  e = own_run(c, st, hp);
  if (e != FMM_OK) return e;
  return hhs_init_batched(c, 1, &c->own_run, &st, hp);
}

extern "C" fmm_status hhs_step(fmm_ctx *c, hhs_state *st, const hhs_params *hp, double dt_top,
                               int64_t stats[3]) {
  fmm_status e = check_params(c, hp);
  if (e != FMM_OK) return e;
  if (!st) return FMM_EINVAL;
  if (st->n < 1 || st->n > c->max_n) return fmm_fail(c, FMM_EINVAL, "state size outside [1, max_n]");
  e = own_run(c, st, hp);
  if (e != FMM_OK) return e;
  return hhs_step_batched(c, 1, &c->own_run, &st, hp, &dt_top, stats);
}

// The comparison integrator of Sec. 2.3: individual (block) timesteps, every
// force evaluation giving the particles whose step ends the acceleration due
// to all the mass, with the particles that are not active where their last
// step left them.  Each tick's solve builds one tree over the whole system
// and evaluates only the active particles as sinks (sink flags: P2P skips
// leaves without one, L2P writes only theirs).
extern "C" fmm_status trad_step(fmm_ctx *c, hhs_state *st, const hhs_params *hp, double dt_top,
                                int64_t stats[3]) {
  fmm_status e = check_params(c, hp);
  if (e != FMM_OK) return e;
  if (!st) return FMM_EINVAL;
  if (st->n < 1 || st->n > c->max_n) return fmm_fail(c, FMM_EINVAL, "state size outside [1, max_n]");
  if (!st->pos || !st->vel || !st->mass || !st->a_old || !st->a_cur || !st->rung)
    return fmm_fail(c, FMM_EINVAL, "NULL state array");
  if (!std::isfinite(dt_top) || dt_top == 0.0) return fmm_fail(c, FMM_EINVAL, "dt_top");
  if (hp->cosmo) return fmm_fail(c, FMM_EINVAL, "trad_step has no comoving form");
  e = own_run(c, st, hp);
  if (e != FMM_OK) return e;
  e = ensure_split_slots(c, 32);
  if (e != FMM_OK) return e;
  hhs_run *r = c->own_run;
  const int64_t n = st->n;
  hipStream_t s = c->stream;
  int64_t calls = 0, parts = 0;
  uint8_t *sinks = r->sinks;  // the run's sink-flag scratch (n bytes)
  auto solve = [&](const uint8_t *flags) {
    ++calls;
    fmm_request q = {st->pos, n, nullptr, n, st->mass, r->acc, r->pot, flags};
    return fmm_forces_batched(c, 1, &q, hp->eps, hp->theta, hp->p);
  };
  // rungs from |a| of an all-particle solve at the start of the top step
  e = solve(nullptr);
  if (e != FMM_OK) return e;
  parts += n;
  hhs_launch_amag(r->acc, n, st->a_cur, st->a_old, s);
  if (!hp->freeze_rungs)
    hhs_launch_rungs(r->all_idx, (int)n, st->a_old, st->a_cur, nullptr, st->rung, dt_top,
                     hp->eta * hp->eps, 0.0, hp->max_levels, s);
  trad_launch_rung_hist(st->rung, n, c->split_cnt, s);
  if (hipMemcpyAsync(c->pin_split, c->split_cnt, sizeof(int32_t) * 32, hipMemcpyDeviceToHost,
                     s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fmm_fail(c, FMM_EDEVICE, "rung readback failed");
  int32_t cnt[32];  // kept for the ticks below, whatever later calls do with the buffer
  std::copy(c->pin_split, c->pin_split + 32, cnt);
  int R = 0;
  for (int k = 0; k < 32; ++k) {
    if (cnt[k] < 0 || (cnt[k] > 0 && k >= hp->max_levels))
      return fmm_fail(c, FMM_EINVAL, "rung outside 0..max_levels-1");
    if (cnt[k] > 0) R = k;
  }
  trad_launch_kick(r->acc, st->rung, n, dt_top, 0, false, st->vel, nullptr, s);  // opening
  const int64_t ticks = (int64_t)1 << R;
  for (int64_t j = 0; j < ticks; ++j) {
    int tz = 0;
    while (!(((j + 1) >> tz) & 1)) ++tz;  // trailing zeros of j + 1
    const int rmin = std::max(0, R - tz);
    trad_launch_drift(st->vel, st->rung, n, dt_top, rmin, st->pos, s);
    trad_launch_flags(st->rung, n, rmin, sinks, s);
    e = solve(rmin > 0 ? sinks : nullptr);
    if (e != FMM_OK) return e;
    for (int k = rmin; k <= R; ++k) parts += cnt[k];
    trad_launch_kick(r->acc, st->rung, n, dt_top, rmin, j + 1 < ticks, st->vel, st->a_cur, s);
  }
  if (hipStreamSynchronize(s) != hipSuccess)
    return fmm_fail(c, FMM_EDEVICE, "trad_step synchronisation failed");
  st->t += dt_top;
  if (stats) {
    stats[0] = calls;
    stats[1] = parts;
    stats[2] = calls;
  }
  c->tree_valid = false;
  return FMM_OK;
}
