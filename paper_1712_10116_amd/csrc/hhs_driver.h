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
