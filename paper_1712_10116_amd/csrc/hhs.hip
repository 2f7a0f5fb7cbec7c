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

// stable partition of sys into slow and fast lists (+ positions within sys);
// pre = exclusive scan of the fast flags; count[0] = number of fast; per
// position i of sys, fflag[i] = 1 when fast and sflag[i] = 1 when slow (the
// sink flags of the two kicks of a KDK half)
__device__ __forceinline__ void split_scatter_at(
    int i, const int32_t *__restrict__ sys, int n_sys, const int32_t *__restrict__ rung, int k,
    const uint32_t *__restrict__ pre, int32_t *__restrict__ slow, int32_t *__restrict__ slow_pos,
    int32_t *__restrict__ fast, int32_t *__restrict__ fast_pos, int32_t *__restrict__ count,
    uint8_t *__restrict__ fflag, uint8_t *__restrict__ sflag) {
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

// Exclusive scan of m uint32 values in place (any m), over tiles of
// SCAN_TILE: the tiles' sums, an exclusive scan of the sums, then each tile's
// own scan plus its offset.  One workgroup of FMM_BLOCK threads per tile (per
// scan for the sums).
#define SCAN_TILE 1024
__device__ __forceinline__ void scan_tile_sum(const uint32_t *v, int m, uint32_t *part, int b) {
  __shared__ uint32_t r[FMM_BLOCK];
  const int base = b * SCAN_TILE;
  uint32_t s = 0;
  for (int i = base + threadIdx.x; i < min(m, base + SCAN_TILE); i += FMM_BLOCK) s += v[i];
  r[threadIdx.x] = s;
  __syncthreads();
  for (int o = FMM_BLOCK / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) r[threadIdx.x] += r[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[b] = r[0];
}

__device__ __forceinline__ void scan_tile_sums(uint32_t *part, int nb) {
  __shared__ uint32_t v[FMM_BLOCK];
  uint32_t run = 0;
  for (int base = 0; base < nb; base += FMM_BLOCK) {
    int i = base + threadIdx.x;
    uint32_t x = i < nb ? part[i] : 0u;
    v[threadIdx.x] = x;
    __syncthreads();
    for (int off = 1; off < FMM_BLOCK; off <<= 1) {
      uint32_t y = threadIdx.x >= off ? v[threadIdx.x - off] : 0u;
      __syncthreads();
      v[threadIdx.x] += y;
      __syncthreads();
    }
    if (i < nb) part[i] = run + v[threadIdx.x] - x;
    run += v[FMM_BLOCK - 1];
    __syncthreads();
  }
}

__device__ __forceinline__ void scan_tile_down(uint32_t *v, int m, const uint32_t *part, int b) {
  __shared__ uint32_t w[FMM_BLOCK];
  const int base = b * SCAN_TILE + threadIdx.x * 4;
  uint32_t x[4], s = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    x[k] = base + k < m ? v[base + k] : 0u;
    s += x[k];
  }
  w[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < FMM_BLOCK; off <<= 1) {
    uint32_t y = threadIdx.x >= off ? w[threadIdx.x - off] : 0u;
    __syncthreads();
    w[threadIdx.x] += y;
    __syncthreads();
  }
  uint32_t run = part[b] + w[threadIdx.x] - s;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (base + k < m) v[base + k] = run;
    run += x[k];
  }
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

// out[p] = mass[p] for the slow particles of a joint set, 0 for the fast ones
// (fflag per position of the joint set)
__global__ __launch_bounds__(FMM_BLOCK) void k_masked_mass_batched(HhsMaskBatch B) {
  const int w = batch_item(B.blk0, B.count, blockIdx.x);
  const HhsMaskItem &M = B.it[w];
  const int i = (blockIdx.x - B.blk0[w]) * FMM_BLOCK + threadIdx.x;
  if (i >= M.n_sys) return;
  const int p = M.sys[i];
  M.out[p] = M.fflag[i] ? 0.0 : M.mass[p];
}

// Rungs (when asked) and the stable slow/fast split of one joint set per
// workgroup: per tile, each thread's fast flag, the tile's exclusive scan
// (wave ballots, then the waves' totals), and the scatter with the fast count
// of the earlier tiles carried along.  The same outputs as the five
// multi-workgroup launches of hhs_launch_big_splits.
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

// Joint sets beyond one workgroup's reach: the multi-workgroup split (rung
// assignment fused with the fast flags, the tiled scan, the scatter) of up
// to HHS_BATCH systems per launch.  Element kernels: block b serves item w
// with eblk0[w] <= b < eblk0[w + 1] (blocks of FMM_BLOCK elements); tile
// kernels likewise over tblk0 (tiles of SCAN_TILE elements); the tile sums
// of item w are scanned by block w.
__global__ __launch_bounds__(FMM_BLOCK) void k_bigsplit_flags(HhsBigSplitBatch B) {
  const int w = batch_item(B.eblk0, B.count, blockIdx.x);
  const HhsSplitItem &S = B.it[w];
  const int i = (blockIdx.x - B.eblk0[w]) * FMM_BLOCK + threadIdx.x;
  if (i >= S.n_sys) return;
  const int p = S.sys[i];
  int r;
  if (S.do_rungs) {
    r = rung_of(p, S.a_old, S.a_cur, S.a_tot, S.dt_top, S.eta_eps, S.eta1_eps, S.max_levels);
    S.rung[p] = r;
  } else {
    r = S.rung[p];
  }
  B.flag[w][i] = r > S.k ? 1u : 0u;
}

__global__ __launch_bounds__(FMM_BLOCK) void k_bigsplit_reduce(HhsBigSplitBatch B) {
  const int w = batch_item(B.tblk0, B.count, blockIdx.x);
  scan_tile_sum(B.flag[w], B.it[w].n_sys, B.part[w], blockIdx.x - B.tblk0[w]);
}

__global__ __launch_bounds__(FMM_BLOCK) void k_bigsplit_partials(HhsBigSplitBatch B) {
  const int w = blockIdx.x;
  scan_tile_sums(B.part[w], B.tblk0[w + 1] - B.tblk0[w]);
}

__global__ __launch_bounds__(FMM_BLOCK) void k_bigsplit_down(HhsBigSplitBatch B) {
  const int w = batch_item(B.tblk0, B.count, blockIdx.x);
  scan_tile_down(B.flag[w], B.it[w].n_sys, B.part[w], blockIdx.x - B.tblk0[w]);
}

__global__ __launch_bounds__(FMM_BLOCK) void k_bigsplit_scatter(HhsBigSplitBatch B) {
  const int w = batch_item(B.eblk0, B.count, blockIdx.x);
  const HhsSplitItem &S = B.it[w];
  const int i = (blockIdx.x - B.eblk0[w]) * FMM_BLOCK + threadIdx.x;
  if (i < S.n_sys)
    split_scatter_at(i, S.sys, S.n_sys, S.rung, S.k, B.flag[w], S.slow, S.slow_pos, S.fast,
                     S.fast_pos, S.count, S.fflag, S.sflag);
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

void hhs_launch_masked_masses(const HhsMaskItem *items, int n_items, hipStream_t s) {
  HhsMaskBatch B;
  B.count = 0;
  B.blk0[0] = 0;
  auto flush = [&]() {
    if (B.count > 0)
      hipLaunchKernelGGL(k_masked_mass_batched, dim3(B.blk0[B.count]), dim3(FMM_BLOCK), 0, s, B);
    B.count = 0;
  };
  for (int j = 0; j < n_items; ++j) {
    if (items[j].n_sys <= 0) continue;
    B.it[B.count] = items[j];
    B.blk0[B.count + 1] = B.blk0[B.count] + (items[j].n_sys + FMM_BLOCK - 1) / FMM_BLOCK;
    if (++B.count == HHS_BATCH) flush();
  }
  flush();
}

void hhs_launch_big_splits(const HhsSplitItem *items, uint32_t *const *flags,
                           uint32_t *const *parts, int n_items, hipStream_t s) {
  HhsBigSplitBatch B;
  B.count = 0;
  B.eblk0[0] = B.tblk0[0] = 0;
  auto flush = [&]() {
    if (B.count == 0) return;
    const dim3 eg(B.eblk0[B.count]), tg(B.tblk0[B.count]), blk(FMM_BLOCK);
    hipLaunchKernelGGL(k_bigsplit_flags, eg, blk, 0, s, B);
    hipLaunchKernelGGL(k_bigsplit_reduce, tg, blk, 0, s, B);
    hipLaunchKernelGGL(k_bigsplit_partials, dim3(B.count), blk, 0, s, B);
    hipLaunchKernelGGL(k_bigsplit_down, tg, blk, 0, s, B);
    hipLaunchKernelGGL(k_bigsplit_scatter, eg, blk, 0, s, B);
    B.count = 0;
  };
  for (int j = 0; j < n_items; ++j) {
    const int m = items[j].n_sys;
    if (m <= 0) continue;
    B.it[B.count] = items[j];
    B.flag[B.count] = flags[j];
    B.part[B.count] = parts[j];
    B.eblk0[B.count + 1] = B.eblk0[B.count] + (m + FMM_BLOCK - 1) / FMM_BLOCK;
    B.tblk0[B.count + 1] = B.tblk0[B.count] + (m + SCAN_TILE - 1) / SCAN_TILE;
    if (++B.count == HHS_BATCH) flush();
  }
  flush();
}
