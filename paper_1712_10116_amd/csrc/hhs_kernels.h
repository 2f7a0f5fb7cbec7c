// Launchers of the HHS and reduction kernels (hhs.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// a_tot NULL: the bound of Eq. 9 is off
void hhs_launch_rungs(const int32_t *sys, int n_sys, const double *a_old, const double *a_cur,
                      const double *a_tot, int32_t *rung, double dt_top, double eta_eps,
                      double eta1_eps, int max_levels, hipStream_t s);
// out[sys[q]] = |a| of row q of acc (SoA, n_sys rows)
void hhs_launch_norm_at(const int32_t *sys, int n_sys, const double *acc, double *out,
                        hipStream_t s);
void hhs_launch_iota(int32_t *v, int n, hipStream_t s);
void hhs_launch_amag(const double *acc, int64_t n, double *a_cur, double *a_old, hipStream_t s);
// Individual-timestep integrator: cnt[k] = particles on rung k (32 ints,
// cleared first); kick (v += a h, twice when asked, h half the particle's
// step, |a| into amag if not NULL) and drift (x += v dt) of the particles with
// rung >= rmin.
void trad_launch_rung_hist(const int32_t *rung, int64_t n, int32_t *cnt, hipStream_t s);
void trad_launch_kick(const double *acc, const int32_t *rung, int64_t n, double dt_top, int rmin,
                      bool twice, double *vel, double *amag, hipStream_t s);
void trad_launch_drift(const double *vel, const int32_t *rung, int64_t n, double dt_top, int rmin,
                       double *pos, hipStream_t s);
// flag[i] = rung[i] >= rmin (the sinks of a tick)
void trad_launch_flags(const int32_t *rung, int64_t n, int rmin, uint8_t *flag, hipStream_t s);
// out[0] = min_i (a[i] + b[i]) over n >= 1 values; part holds
// min(1024, ceil(n / 256)) doubles of scratch
void hhs_launch_min_sum(const double *a, const double *b, int64_t n, double *part, double *out,
                        hipStream_t s);
// Blocks of the invariant reduction: each writes 12 FP64 partial sums to
// part[block * 12 + k], which are then added in block order.
#define FMM_INV_BLOCKS 512
void launch_invariants(const double *pos, const double *vel, const double *mass,
                       const double *acc, const double *pot, int64_t n, double *part, int nblk,
                       hipStream_t s);

// Batched launches: the kicks, drifts, masked masses or rung assignments +
// splits of many systems (items with an empty set are skipped), HHS_BATCH
// systems per launch.
// Kick: vel[p] += acc[q] dt for p = set[i], q = setpos[i] (acc SoA with
// n_joint rows, vel with n), and amag[p] = |acc[q]| when amag is not NULL.
// Drift: pos[p] += vel[p] dt for p = set[i].  Split: the rung assignment
// (when do_rungs; the rule of hhs_launch_rungs) and the stable slow/fast
// split of one joint set at rung k; one workgroup per set up to
// HHS_SPLIT_MAX_N, the multi-workgroup launches of hhs_launch_big_splits
// beyond.
#define HHS_BATCH 16
#define HHS_SPLIT_MAX_N 16384
struct HhsKickItem {
  const int32_t *set, *setpos;
  const double *acc;
  double *vel, *amag;
  int64_t n_joint, n;
  double dt;
  int n_set;
};
struct HhsDriftItem {
  const int32_t *set;
  const double *vel;
  double *pos;
  int64_t n;
  double dt;
  int n_set;
};
struct HhsSplitItem {
  const int32_t *sys;
  int32_t *rung;
  const double *a_old, *a_cur, *a_tot;
  int32_t *slow, *slow_pos, *fast, *fast_pos, *count;
  uint8_t *fflag, *sflag;
  double dt_top, eta_eps, eta1_eps;
  int n_sys, k, max_levels, do_rungs;
};
struct HhsKickBatch {
  HhsKickItem it[HHS_BATCH];
  int blk0[HHS_BATCH + 1];
  int count;
};
struct HhsDriftBatch {
  HhsDriftItem it[HHS_BATCH];
  int blk0[HHS_BATCH + 1];
  int count;
};
struct HhsSplitBatch {
  HhsSplitItem it[HHS_BATCH];
  int count;
};
// Splits of joint sets beyond HHS_SPLIT_MAX_N: the split items plus each
// system's flag (n_sys) and tile-sum (n_sys / 1024 + 1) scratch.
struct HhsBigSplitBatch {
  HhsSplitItem it[HHS_BATCH];
  uint32_t *flag[HHS_BATCH], *part[HHS_BATCH];
  int eblk0[HHS_BATCH + 1], tblk0[HHS_BATCH + 1];
  int count;
};
// by-value kernel arguments stay within the 4 KiB that a launch carries
static_assert(sizeof(HhsBigSplitBatch) <= 4096 && sizeof(HhsSplitBatch) <= 4096,
              "batch exceeds the kernel argument space");
// Masked masses of kickS2F: out[sys[i]] = 0 where fflag[i], else mass[sys[i]]
// (the rest of out untouched).
struct HhsMaskItem {
  const int32_t *sys;
  const uint8_t *fflag;
  const double *mass;
  double *out;
  int n_sys;
};
struct HhsMaskBatch {
  HhsMaskItem it[HHS_BATCH];
  int blk0[HHS_BATCH + 1];
  int count;
};
void hhs_launch_kicks(const HhsKickItem *items, int n_items, hipStream_t s);
void hhs_launch_drifts(const HhsDriftItem *items, int n_items, hipStream_t s);
void hhs_launch_splits(const HhsSplitItem *items, int n_items, hipStream_t s);
void hhs_launch_masked_masses(const HhsMaskItem *items, int n_items, hipStream_t s);
void hhs_launch_big_splits(const HhsSplitItem *items, uint32_t *const *flags,
                           uint32_t *const *parts, int n_items, hipStream_t s);
