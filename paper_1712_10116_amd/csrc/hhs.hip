// Device kernels of the HHS integrator (Sec. 2.2, Algorithms 1-3) and the
// FP64 conservation reductions.  The host walks the EVOLVE_HOLD recursion;
// every per-particle step (rung assignment, slow/fast split, mass masking of
// the fast system for kickS2F, kicks, drifts) runs here in FP64.
#include <algorithm>

#include "common.h"
#include "hhs_kernels.h"

// rung = smallest k with dt_top 2^-k <= sqrt(eta eps / a), a = |a_old| + |a_cur|,
// decided as (dt_k dt_k) a <= eta eps (no square root), clamped to L-1; with
// a_tot (Eq. 9) the rung must also satisfy (dt_k dt_k) |a|_tot <= eta1 eps
__device__ __forceinline__ int rung_of(int p, const double *__restrict__ a_old,
                                       const double *__restrict__ a_cur,
                                       const double *__restrict__ a_tot, double dt_top,
                                       double eta_eps, double eta1_eps, int max_levels) {
  double a = a_old[p] + a_cur[p];
  const double at = a_tot ? a_tot[p] : 0.0;
  int r = max_levels - 1;
  for (int k = max_levels - 1; k >= 0; --k) {
    double dtk = ldexp(dt_top, -k);
    bool ok = (dtk * dtk) * a <= eta_eps;
    if (a_tot) ok = ok && (dtk * dtk) * at <= eta1_eps;
    if (ok) r = k;
  }
  return r;
}

__global__ __launch_bounds__(FMM_BLOCK) void k_rungs(const int32_t *__restrict__ sys, int n_sys,
                                                     const double *__restrict__ a_old,
                                                     const double *__restrict__ a_cur,
                                                     const double *__restrict__ a_tot,
                                                     int32_t *__restrict__ rung, double dt_top,
                                                     double eta_eps, double eta1_eps,
                                                     int max_levels) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_sys) return;
  const int p = sys[i];
  rung[p] = rung_of(p, a_old, a_cur, a_tot, dt_top, eta_eps, eta1_eps, max_levels);
}

// out[sys[q]] = |a| of row q of a joint-set acceleration (SoA, n_sys rows)
__global__ __launch_bounds__(FMM_BLOCK) void k_norm_at(const int32_t *__restrict__ sys,
                                                       int n_sys, const double *__restrict__ acc,
                                                       double *__restrict__ out) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_sys) return;
  const double ax = acc[q], ay = acc[n_sys + q], az = acc[2 * n_sys + q];
  out[sys[q]] = sqrt(ax * ax + ay * ay + az * az);
}

// flag[i] = 1 if sys[i] is fast at rung k (rung > k)
__global__ __launch_bounds__(FMM_BLOCK) void k_fast_flags(const int32_t *__restrict__ sys, int n_sys,
                                                          const int32_t *__restrict__ rung, int k,
                                                          uint32_t *__restrict__ flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_sys) return;
  flag[i] = rung[sys[i]] > k ? 1u : 0u;
}

// stable partition of sys into slow and fast lists (+ positions within sys);
// pre = exclusive scan of the fast flags; count[0] = number of fast; per
// position i of sys, fflag[i] = 1 when fast and sflag[i] = 1 when slow (the
// sink flags of the two kicks of a KDK half)
__global__ __launch_bounds__(FMM_BLOCK) void k_split_scatter(
    const int32_t *__restrict__ sys, int n_sys, const int32_t *__restrict__ rung, int k,
    const uint32_t *__restrict__ pre, int32_t *__restrict__ slow, int32_t *__restrict__ slow_pos,
    int32_t *__restrict__ fast, int32_t *__restrict__ fast_pos, int32_t *__restrict__ count,
    uint8_t *__restrict__ fflag, uint8_t *__restrict__ sflag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_sys) return;
  int p = sys[i];
  int f = (int)pre[i];
  const bool is_fast = rung[p] > k;
  if (is_fast) {
    fast[f] = p;
    fast_pos[f] = i;
  } else {
    slow[i - f] = p;
    slow_pos[i - f] = i;
  }
  fflag[i] = is_fast ? 1 : 0;
  sflag[i] = is_fast ? 0 : 1;
  if (i == n_sys - 1) count[0] = f + (is_fast ? 1 : 0);
}

// out[p] = mass[p] for the slow particles of the joint set sys, 0 for the
// fast ones (fflag per position of sys)
__global__ __launch_bounds__(FMM_BLOCK) void k_masked_mass(const int32_t *__restrict__ sys,
                                                           int n_sys,
                                                           const uint8_t *__restrict__ fflag,
                                                           const double *__restrict__ mass,
                                                           double *__restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_sys) return;
  const int p = sys[i];
  out[p] = fflag[i] ? 0.0 : mass[p];
}

__global__ __launch_bounds__(FMM_BLOCK) void k_iota(int32_t *__restrict__ v, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = i;
}

__global__ __launch_bounds__(FMM_BLOCK) void k_amag(const double *__restrict__ acc, int64_t n,
                                                    double *__restrict__ a_cur,
                                                    double *__restrict__ a_old) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double ax = acc[i], ay = acc[n + i], az = acc[2 * n + i];
  a_cur[i] = sqrt(ax * ax + ay * ay + az * az);
  a_old[i] = 0.0;
}

// Individual-timestep integrator (Sec. 2.3): particle i steps with
// dt_top 2^-rung[i]; the kick and drift kernels act on the particles with
// rung >= rmin, the ones whose step ends at the current tick.  The histogram
// counts rungs 0..30 and puts any other value in bucket 31.
__global__ __launch_bounds__(FMM_BLOCK) void k_rung_hist(const int32_t *__restrict__ rung,
                                                         int64_t n, int32_t *__restrict__ cnt) {
  __shared__ int32_t h[32];
  if (threadIdx.x < 32) h[threadIdx.x] = 0;
  __syncthreads();
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const int r = rung[i];
    atomicAdd(&h[r >= 0 && r <= 30 ? r : 31], 1);  // 31: outside every valid rung range
  }
  __syncthreads();
  if (threadIdx.x < 32 && h[threadIdx.x]) atomicAdd(&cnt[threadIdx.x], h[threadIdx.x]);
}

// v += a h (h = half of the particle's step), and again when twice is set
// (the closing half kick of one step followed by the opening one of the
// next); |a| into amag when given
__global__ __launch_bounds__(FMM_BLOCK) void k_rung_kick(const double *__restrict__ acc,
                                                         const int32_t *__restrict__ rung,
                                                         int64_t n, double dt_top, int rmin,
                                                         bool twice, double *__restrict__ vel,
                                                         double *__restrict__ amag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int r = rung[i];
  if (r < rmin) return;
  const double h = ldexp(dt_top, -r) * 0.5;
  const double ax = acc[i], ay = acc[n + i], az = acc[2 * n + i];
  double vx = vel[i] + ax * h, vy = vel[n + i] + ay * h, vz = vel[2 * n + i] + az * h;
  if (twice) {
    vx += ax * h;
    vy += ay * h;
    vz += az * h;
  }
  vel[i] = vx;
  vel[n + i] = vy;
  vel[2 * n + i] = vz;
  if (amag) amag[i] = sqrt(ax * ax + ay * ay + az * az);
}

// flag[i] = 1 for the particles whose step ends at the tick (rung >= rmin)
__global__ __launch_bounds__(FMM_BLOCK) void k_rung_flags(const int32_t *__restrict__ rung,
                                                          int64_t n, int rmin,
                                                          uint8_t *__restrict__ flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[i] = rung[i] >= rmin ? 1 : 0;
}

__global__ __launch_bounds__(FMM_BLOCK) void k_rung_drift(const double *__restrict__ vel,
                                                          const int32_t *__restrict__ rung,
                                                          int64_t n, double dt_top, int rmin,
                                                          double *__restrict__ pos) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int r = rung[i];
  if (r < rmin) return;
  const double dt = ldexp(dt_top, -r);
  pos[i] += vel[i] * dt;
  pos[n + i] += vel[n + i] * dt;
  pos[2 * n + i] += vel[2 * n + i] * dt;
}

// block minima of a[i] + b[i] (grid-stride), then one block reduces them
__global__ __launch_bounds__(FMM_BLOCK) void k_min_sum_partial(const double *__restrict__ a,
                                                               const double *__restrict__ b,
                                                               int64_t n, double *__restrict__ part) {
  double m = INFINITY;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    m = fmin(m, a[i] + b[i]);
  __shared__ double red[FMM_BLOCK];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = FMM_BLOCK / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(FMM_BLOCK) void k_min_final(const double *__restrict__ part, int nb,
                                                         double *__restrict__ out) {
  double m = INFINITY;
  for (int i = threadIdx.x; i < nb; i += FMM_BLOCK) m = fmin(m, part[i]);
  __shared__ double red[FMM_BLOCK];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = FMM_BLOCK / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// per-block FP64 partial sums of the 12 invariants; the host adds the blocks
// in a fixed order
__global__ __launch_bounds__(FMM_BLOCK) void k_invariants(const double *__restrict__ pos,
                                                          const double *__restrict__ vel,
                                                          const double *__restrict__ mass,
                                                          const double *__restrict__ acc,
                                                          const double *__restrict__ pot,
                                                          int64_t n, double *__restrict__ part) {
  double s[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) s[k] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double m = mass ? mass[i] : 1.0;
    if (acc) {
      double ax = acc[i], ay = acc[n + i], az = acc[2 * n + i];
      s[0] += m * ax;
      s[1] += m * ay;
      s[2] += m * az;
      s[11] += m * sqrt(ax * ax + ay * ay + az * az);
    }
    if (vel) {
      double vx = vel[i], vy = vel[n + i], vz = vel[2 * n + i];
      s[3] += m * vx;
      s[4] += m * vy;
      s[5] += m * vz;
      s[9] += 0.5 * m * (vx * vx + vy * vy + vz * vz);
      if (pos) {
        double x = pos[i], y = pos[n + i], z = pos[2 * n + i];
        s[6] += m * (y * vz - z * vy);
        s[7] += m * (z * vx - x * vz);
        s[8] += m * (x * vy - y * vx);
      }
    }
    if (pot) s[10] += 0.5 * m * pot[i];
  }
  __shared__ double red[FMM_BLOCK];
  for (int k = 0; k < 12; ++k) {
    red[threadIdx.x] = s[k];
    __syncthreads();
    for (int o = FMM_BLOCK / 2; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x * 12 + k] = red[0];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// The per-system kernels of many systems in one launch.  The arguments of at
// most HHS_BATCH systems travel by value in the kernel's argument block.
// Kicks and drifts: block b serves item w with blk0[w] <= b < blk0[w + 1]
// (running counts of each item's blocks of FMM_BLOCK elements), so a block
// stays inside one system's range.  Rungs and split: one workgroup per
// system, which walks its joint set in tiles of SPLIT_THREADS.

__device__ __forceinline__ int batch_item(const int *blk0, int count, int b) {
  int w = 0;
  while (w + 1 < count && blk0[w + 1] <= b) ++w;
  return w;
}

__global__ __launch_bounds__(FMM_BLOCK) void k_kick_batched(HhsKickBatch B) {
  const int w = batch_item(B.blk0, B.count, blockIdx.x);
  const HhsKickItem &K = B.it[w];
  const int i = (blockIdx.x - B.blk0[w]) * FMM_BLOCK + threadIdx.x;
  if (i >= K.n_set) return;
  const int p = K.set[i], q = K.setpos[i];
  const int64_t nj = K.n_joint, n = K.n;
  const double ax = K.acc[q], ay = K.acc[nj + q], az = K.acc[2 * nj + q];
  K.vel[p] += ax * K.dt;
  K.vel[n + p] += ay * K.dt;
  K.vel[2 * n + p] += az * K.dt;
  if (K.amag) K.amag[p] = sqrt(ax * ax + ay * ay + az * az);
}

__global__ __launch_bounds__(FMM_BLOCK) void k_drift_batched(HhsDriftBatch B) {
  const int w = batch_item(B.blk0, B.count, blockIdx.x);
  const HhsDriftItem &D = B.it[w];
  const int i = (blockIdx.x - B.blk0[w]) * FMM_BLOCK + threadIdx.x;
  if (i >= D.n_set) return;
  const int p = D.set[i];
  const int64_t n = D.n;
  D.pos[p] += D.vel[p] * D.dt;
  D.pos[n + p] += D.vel[n + p] * D.dt;
  D.pos[2 * n + p] += D.vel[2 * n + p] * D.dt;
}

// Rungs (when asked) and the stable slow/fast split of one joint set per
// workgroup: per tile, each thread's fast flag, the tile's exclusive scan
// (wave ballots, then the waves' totals), and the scatter with the fast count
// of the earlier tiles carried along.  The same outputs as hhs_launch_rungs
// followed by hhs_launch_split.
#define SPLIT_THREADS 1024
__global__ __launch_bounds__(SPLIT_THREADS) void k_split_batched(HhsSplitBatch B) {
  __shared__ int wtot[SPLIT_THREADS / 64];
  const HhsSplitItem &S = B.it[blockIdx.x];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const unsigned long long below = lanes_below_mask();
  int carry = 0;
  for (int base = 0; base < S.n_sys; base += SPLIT_THREADS) {
    const int i = base + tid;
    const bool valid = i < S.n_sys;
    int p = 0;
    bool fast = false;
    if (valid) {
      p = S.sys[i];
      int r;
      if (S.do_rungs) {
        r = rung_of(p, S.a_old, S.a_cur, S.a_tot, S.dt_top, S.eta_eps, S.eta1_eps,
                    S.max_levels);
        S.rung[p] = r;
      } else {
        r = S.rung[p];
      }
      fast = r > S.k;
    }
    const unsigned long long bal = __ballot(fast);
    if (lane == 0) wtot[w] = __popcll(bal);
    __syncthreads();
    int before = carry, total = 0;
    for (int v = 0; v < SPLIT_THREADS / 64; ++v) {
      before += v < w ? wtot[v] : 0;
      total += wtot[v];
    }
    if (valid) {
      const int f = before + __popcll(bal & below);  // fast ones before element i
      if (fast) {
        S.fast[f] = p;
        S.fast_pos[f] = i;
      } else {
        S.slow[i - f] = p;
        S.slow_pos[i - f] = i;
      }
      S.fflag[i] = fast ? 1 : 0;
      S.sflag[i] = fast ? 0 : 1;
    }
    carry += total;
    __syncthreads();  // wtot is rewritten by the next tile
  }
  if (tid == 0) S.count[0] = carry;
}

#define NB(n) dim3((unsigned)(((n) + FMM_BLOCK - 1) / FMM_BLOCK))

void hhs_launch_rungs(const int32_t *sys, int n_sys, const double *a_old, const double *a_cur,
                      const double *a_tot, int32_t *rung, double dt_top, double eta_eps,
                      double eta1_eps, int max_levels, hipStream_t s) {
  if (n_sys > 0)
    hipLaunchKernelGGL(k_rungs, NB(n_sys), dim3(FMM_BLOCK), 0, s, sys, n_sys, a_old, a_cur, a_tot,
                       rung, dt_top, eta_eps, eta1_eps, max_levels);
}

void hhs_launch_norm_at(const int32_t *sys, int n_sys, const double *acc, double *out,
                        hipStream_t s) {
  if (n_sys > 0)
    hipLaunchKernelGGL(k_norm_at, NB(n_sys), dim3(FMM_BLOCK), 0, s, sys, n_sys, acc, out);
}

void hhs_launch_split(const int32_t *sys, int n_sys, const int32_t *rung, int k, uint32_t *flag,
                      uint32_t *scan_part, int32_t *slow, int32_t *slow_pos, int32_t *fast,
                      int32_t *fast_pos, int32_t *count, uint8_t *fflag, uint8_t *sflag,
                      hipStream_t s) {
  if (n_sys <= 0) return;
  hipLaunchKernelGGL(k_fast_flags, NB(n_sys), dim3(FMM_BLOCK), 0, s, sys, n_sys, rung, k, flag);
  hhs_launch_scan_u32(flag, n_sys, scan_part, s);
  hipLaunchKernelGGL(k_split_scatter, NB(n_sys), dim3(FMM_BLOCK), 0, s, sys, n_sys, rung, k, flag,
                     slow, slow_pos, fast, fast_pos, count, fflag, sflag);
}

void hhs_launch_masked_mass(const int32_t *sys, int n_sys, const uint8_t *fflag,
                            const double *mass, double *out, hipStream_t s) {
  if (n_sys > 0)
    hipLaunchKernelGGL(k_masked_mass, NB(n_sys), dim3(FMM_BLOCK), 0, s, sys, n_sys, fflag, mass,
                       out);
}

void hhs_launch_iota(int32_t *v, int n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_iota, NB(n), dim3(FMM_BLOCK), 0, s, v, n);
}

void hhs_launch_amag(const double *acc, int64_t n, double *a_cur, double *a_old, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_amag, NB(n), dim3(FMM_BLOCK), 0, s, acc, n, a_cur, a_old);
}

void trad_launch_rung_hist(const int32_t *rung, int64_t n, int32_t *cnt, hipStream_t s) {
  hipMemsetAsync(cnt, 0, 32 * sizeof(int32_t), s);
  if (n > 0) hipLaunchKernelGGL(k_rung_hist, NB(n), dim3(FMM_BLOCK), 0, s, rung, n, cnt);
}

void trad_launch_kick(const double *acc, const int32_t *rung, int64_t n, double dt_top, int rmin,
                      bool twice, double *vel, double *amag, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_rung_kick, NB(n), dim3(FMM_BLOCK), 0, s, acc, rung, n, dt_top, rmin,
                       twice, vel, amag);
}

void trad_launch_flags(const int32_t *rung, int64_t n, int rmin, uint8_t *flag, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_rung_flags, NB(n), dim3(FMM_BLOCK), 0, s, rung, n, rmin, flag);
}

void trad_launch_drift(const double *vel, const int32_t *rung, int64_t n, double dt_top, int rmin,
                       double *pos, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_rung_drift, NB(n), dim3(FMM_BLOCK), 0, s, vel, rung, n, dt_top, rmin,
                       pos);
}

void hhs_launch_min_sum(const double *a, const double *b, int64_t n, double *part, double *out,
                        hipStream_t s) {
  if (n <= 0) return;
  const int nb = (int)std::min<int64_t>(1024, (n + FMM_BLOCK - 1) / FMM_BLOCK);
  hipLaunchKernelGGL(k_min_sum_partial, dim3(nb), dim3(FMM_BLOCK), 0, s, a, b, n, part);
  hipLaunchKernelGGL(k_min_final, dim3(1), dim3(FMM_BLOCK), 0, s, part, nb, out);
}

void launch_invariants(const double *pos, const double *vel, const double *mass,
                       const double *acc, const double *pot, int64_t n, double *part, int nblk,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_invariants, dim3(nblk), dim3(FMM_BLOCK), 0, s, pos, vel, mass, acc, pot, n,
                     part);
}

void hhs_launch_kicks(const HhsKickItem *items, int n_items, hipStream_t s) {
  HhsKickBatch B;
  B.count = 0;
  B.blk0[0] = 0;
  auto flush = [&]() {
    if (B.count > 0)
      hipLaunchKernelGGL(k_kick_batched, dim3(B.blk0[B.count]), dim3(FMM_BLOCK), 0, s, B);
    B.count = 0;
  };
  for (int j = 0; j < n_items; ++j) {
    if (items[j].n_set <= 0) continue;
    B.it[B.count] = items[j];
    B.blk0[B.count + 1] = B.blk0[B.count] + (items[j].n_set + FMM_BLOCK - 1) / FMM_BLOCK;
    if (++B.count == HHS_BATCH) flush();
  }
  flush();
}

void hhs_launch_drifts(const HhsDriftItem *items, int n_items, hipStream_t s) {
  HhsDriftBatch B;
  B.count = 0;
  B.blk0[0] = 0;
  auto flush = [&]() {
    if (B.count > 0)
      hipLaunchKernelGGL(k_drift_batched, dim3(B.blk0[B.count]), dim3(FMM_BLOCK), 0, s, B);
    B.count = 0;
  };
  for (int j = 0; j < n_items; ++j) {
    if (items[j].n_set <= 0) continue;
    B.it[B.count] = items[j];
    B.blk0[B.count + 1] = B.blk0[B.count] + (items[j].n_set + FMM_BLOCK - 1) / FMM_BLOCK;
    if (++B.count == HHS_BATCH) flush();
  }
  flush();
}

void hhs_launch_splits(const HhsSplitItem *items, int n_items, hipStream_t s) {
  HhsSplitBatch B;
  B.count = 0;
  auto flush = [&]() {
    if (B.count > 0)
      hipLaunchKernelGGL(k_split_batched, dim3(B.count), dim3(SPLIT_THREADS), 0, s, B);
    B.count = 0;
  };
  for (int j = 0; j < n_items; ++j) {
    if (items[j].n_sys <= 0) continue;
    B.it[B.count] = items[j];
    if (++B.count == HHS_BATCH) flush();
  }
  flush();
}
