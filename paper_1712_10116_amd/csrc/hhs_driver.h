// Internal entry points of the HHS driver used by the request server.
#pragma once
#include "context.h"

// hhs_run_create with the run's arrays carved from mem (hhs_run_bytes bytes of
// device memory owned by the caller), or its own block when mem is NULL.
fmm_status hhs_run_create_at(fmm_ctx *c, int64_t n, int max_levels, void *mem, hhs_run **out);

// hhs_step_batched that also reports, per system i, sys_stats[2i] force
// evaluations and sys_stats[2i+1] their active particles (sys_stats may be NULL).
fmm_status hhs_step_batched_ex(fmm_ctx *c, int n_sys, hhs_run *const *runs,
                               hhs_state *const *states, const hhs_params *hp,
                               const double *dt_top, int64_t stats[3], int64_t *sys_stats);

// out[0] (device) = min over the state's particles of |a_old| + |a_cur|,
// stream ordered on the run's context.
void hhs_run_launch_min_amag(hhs_run *r, const hhs_state *st, double *out);

// Round-by-round driving of many systems (the request server's continuous
// batching).  A system's top-level step is a frame stack that persists
// between rounds; a round advances every running system until it waits on
// the device or ends its step (hhs_sys_advance), then serves either every
// pending split count in one readback or every pending KDK half in batched
// launches (hhs_sys_serve; *served false when nothing waits).  Each system
// follows exactly the operations of a step of it alone, whatever the others
// are doing.  slot is the system's split counter, distinct among the systems
// of one call; hhs_sys_begin needs an idle system (no step in progress) and
// starts a step of dt_top at st->t, which the caller advances once
// hhs_sys_idle reports the step ended.
struct HhsSys;
HhsSys *hhs_sys_create(hhs_run *run, hhs_state *st, int slot);
void hhs_sys_destroy(HhsSys *s);
void hhs_sys_begin(HhsSys *s, double dt_top);
bool hhs_sys_idle(const HhsSys *s);
void hhs_sys_counts(const HhsSys *s, int64_t *kicks, int64_t *parts);
fmm_status hhs_sys_advance(fmm_ctx *c, HhsSys *const *sys, int n_sys, const hhs_params *hp);
fmm_status hhs_sys_serve(fmm_ctx *c, HhsSys *const *sys, int n_sys, const hhs_params *hp,
                         int64_t *kicks, bool *served);
