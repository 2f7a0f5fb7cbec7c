// Morton-ordered oct-tree build on gfx950.
//
// Steps (all device-side; the host only queues launches):
//   1. root box: per-axis min/max of the active positions; centre
//      c = (lo+hi)/2, side L = max extent (1 if zero), origin o = c - L/2,
//      scale s = 2^21/L;
//   2. 63-bit Morton keys from q_d = clamp(floor((x_d - o_d) s), 0, 2^21-1),
//      x bits at 3b+2, y at 3b+1, z at 3b;
//   3. stable LSD radix sort of (key, active slot), 8 passes of 8 bits; ranks
//      inside a wavefront come from 8 ballots per 64 keys;
//   4. top-down split (the paper's recursive build, Sec. 2.3, done level by
//      level): a cell of level l < 21 holding more than leaf_size particles
//      gets one child per non-empty octant of its key range; children of a
//      level are emitted in Morton order after a count / scan / emit sweep;
//   5. geometric centre z = o + (i + 1/2) L 2^-l and half side h = L 2^-(l+1)
//      of every cell; cell-local FP32 offsets of every particle.
// All decisions are the same IEEE double expressions as in the definition
// above, built with -ffp-contract=off, so keys, octant membership and centres
// are reproducible bit for bit.
#include <algorithm>

#include "common.h"
#include "hhs_kernels.h"

#define SORT_WAVES 16                          // wavefronts per radix tile
#define SORT_ITEMS (SORT_TILE / (SORT_WAVES * 64))
#define SORT_THREADS (SORT_WAVES * 64)
#define SMALL_ITEMS 16

// ---------------------------------------------------------------------------
// request of every slot (binary search in the request offsets)
// ---------------------------------------------------------------------------

// request of every active slot; also clears the header counters that the
// following kernels accumulate into (non-finite flag, leaf count)
__global__ __launch_bounds__(FMM_BLOCK) void k_slot_req(DevTree t, int n) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s == 0) {
    t.hdr->nonfinite = 0;
    t.hdr->n_leaves = 0;
  }
  if (s < n) t.slot_req[s] = upper_index(t.req_off, t.n_req, s);
}

// ---------------------------------------------------------------------------
// root box of every request
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(FMM_BLOCK) void k_bbox_partial(DevTree t) {
  const int r = upper_index(t.blk_off, t.n_req, blockIdx.x);
  const DevReq q = t.reqs[r];
  const int lb = blockIdx.x - t.blk_off[r], nbr = t.blk_off[r + 1] - t.blk_off[r];
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  int bad = 0;
  for (int i = lb * blockDim.x + threadIdx.x; i < q.n; i += nbr * blockDim.x) {
    int64_t g = q.active ? q.active[i] : i;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double x = q.pos[d * q.n_total + g];
      bad |= !isfinite(x);
      lo[d] = fmin(lo[d], x);
      hi[d] = fmax(hi[d], x);
    }
  }
  __shared__ double red[6][FMM_BLOCK];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    red[d][threadIdx.x] = lo[d];
    red[3 + d][threadIdx.x] = hi[d];
  }
  if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(&t.hdr->nonfinite, 1);
  for (int o = FMM_BLOCK / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        red[d][threadIdx.x] = fmin(red[d][threadIdx.x], red[d][threadIdx.x + o]);
        red[3 + d][threadIdx.x] = fmax(red[3 + d][threadIdx.x], red[3 + d][threadIdx.x + o]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) t.bbox_part[blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// c = (lo+hi)/2, L = max extent (1 if 0), o = c - L/2, s = 2^21/L
__device__ __forceinline__ void finish_box(Box &bx, double lo[3], double hi[3], bool empty) {
  if (empty)
    for (int d = 0; d < 3; ++d) lo[d] = hi[d] = 0.0;
  double c[3], L = 0.0;
  for (int d = 0; d < 3; ++d) {
    c[d] = 0.5 * (lo[d] + hi[d]);
    double e = hi[d] - lo[d];
    if (e > L) L = e;
  }
  if (L == 0.0) L = 1.0;
  for (int d = 0; d < 3; ++d) {
    bx.o[d] = c[d] - 0.5 * L;
    bx.lo[d] = lo[d];
    bx.hi[d] = hi[d];
  }
  bx.L = L;
  bx.s = 2097152.0 / L;
}

// one wavefront per request
__global__ __launch_bounds__(FMM_BLOCK) void k_bbox_final(DevTree t) {
  const int r = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (r >= t.n_req) return;
  const int b0 = t.blk_off[r], b1 = t.blk_off[r + 1];
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int b = b0 + lane; b < b1; b += 64)
    for (int d = 0; d < 3; ++d) {
      lo[d] = fmin(lo[d], t.bbox_part[b * 6 + d]);
      hi[d] = fmax(hi[d], t.bbox_part[b * 6 + 3 + d]);
    }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = fmin(lo[d], __shfl_xor(lo[d], off, 64));
      hi[d] = fmax(hi[d], __shfl_xor(hi[d], off, 64));
    }
  if (lane != 0) return;
  finish_box(t.box[r], lo, hi, t.reqs[r].n == 0);
}

// ---------------------------------------------------------------------------
// Morton keys
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t spread3(uint64_t x) {
  x &= 0x1fffffull;
  x = (x | x << 32) & 0x1f00000000ffffull;
  x = (x | x << 16) & 0x1f0000ff0000ffull;
  x = (x | x << 8) & 0x100f00f00f00f00full;
  x = (x | x << 4) & 0x10c30c30c30c30c3ull;
  x = (x | x << 2) & 0x1249249249249249ull;
  return x;
}

__device__ __forceinline__ uint32_t compact3(uint64_t x) {
  x &= 0x1249249249249249ull;
  x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
  x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
  x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
  x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
  x = (x ^ (x >> 32)) & 0x1fffffull;
  return (uint32_t)x;
}

__device__ __forceinline__ uint64_t quantise(double x, double o, double s) {
  double q = floor((x - o) * s);
  const double qmax = 2097151.0;
  if (!(q >= 0.0)) q = 0.0;
  if (q > qmax) q = qmax;
  return (uint64_t)q;
}

__device__ __forceinline__ void make_key(const DevTree &t, int s, uint64_t *key, int32_t *slot) {
  const int r = t.slot_req[s];
  const DevReq q = t.reqs[r];
  const int i = s - q.off;
  int64_t g = q.active ? q.active[i] : i;
  const Box &bx = t.box[r];
  const double x = q.pos[g], y = q.pos[q.n_total + g], z = q.pos[2 * q.n_total + g];
  uint64_t qx = quantise(x, bx.o[0], bx.s);
  uint64_t qy = quantise(y, bx.o[1], bx.s);
  uint64_t qz = quantise(z, bx.o[2], bx.s);
  key[s] = (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
  slot[s] = s;
  t.pak[s] = make_double4(x, y, z, 0.0);
}

// keys and slots into key2 / slot2 when the sort that follows makes an odd
// number of passes (so that its result lands in key / slot)
__global__ __launch_bounds__(FMM_BLOCK) void k_keys(DevTree t, int n, int odd) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) make_key(t, s, odd ? t.key2 : t.key, odd ? t.slot2 : t.slot);
}

// ---------------------------------------------------------------------------
// stable LSD radix sort, 8-bit digits
// ---------------------------------------------------------------------------
// digit of element i: bits [shift, shift+8) of its key (by_req = 0) or of the
// request of its slot (by_req = 1; these passes come last, so the final order
// is by (request, key, slot))
__device__ __forceinline__ uint32_t sort_digit(const uint64_t *key, const int32_t *slot,
                                               const int32_t *slot_req, int i, int shift,
                                               int by_req) {
  return by_req ? ((uint32_t)slot_req[slot[i]] >> shift) & 255u
                : (uint32_t)(key[i] >> shift) & 255u;
}

// clear_slices > 0: also clears this tile's column of the clear_slices
// histograms that follow hist (one per later raw pass, 256 * nblk apart)
__global__ __launch_bounds__(SORT_THREADS) void k_sort_hist(const uint64_t *__restrict__ key,
                                                            const int32_t *__restrict__ slot,
                                                            const int32_t *__restrict__ slot_req,
                                                            int n, int shift, int by_req,
                                                            uint32_t *__restrict__ hist,
                                                            int nblk, int clear_slices) {
  __shared__ uint32_t h[256];
  if (threadIdx.x < 256) h[threadIdx.x] = 0;
  __syncthreads();
  const int base = blockIdx.x * SORT_TILE;
#pragma unroll
  for (int it = 0; it < SORT_ITEMS; ++it) {
    const int i = base + it * SORT_THREADS + threadIdx.x;
    if (i < n) atomicAdd(&h[sort_digit(key, slot, slot_req, i, shift, by_req)], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 256) {
    hist[threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
    for (int p = 1; p <= clear_slices; ++p)
      hist[(size_t)p * 256 * nblk + threadIdx.x * nblk + blockIdx.x] = 0u;
  }
}

// Per-digit exclusive scan over the blocks: hist[d][0..nblk) in place, digit
// total to dtot[d].  One workgroup per digit, coalesced tiles of 256.
__global__ __launch_bounds__(FMM_BLOCK) void k_sort_digit_scan(uint32_t *hist, int nblk,
                                                               uint32_t *dtot) {
  __shared__ uint32_t v[FMM_BLOCK];
  uint32_t *h = hist + (size_t)blockIdx.x * nblk;
  uint32_t run = 0;
  for (int base = 0; base < nblk; base += FMM_BLOCK) {
    int i = base + threadIdx.x;
    uint32_t x = i < nblk ? h[i] : 0u;
    v[threadIdx.x] = x;
    __syncthreads();
    for (int off = 1; off < FMM_BLOCK; off <<= 1) {
      uint32_t y = threadIdx.x >= off ? v[threadIdx.x - off] : 0u;
      __syncthreads();
      v[threadIdx.x] += y;
      __syncthreads();
    }
    if (i < nblk) h[i] = run + v[threadIdx.x] - x;
    run += v[FMM_BLOCK - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) dtot[blockIdx.x] = run;
}

// Exclusive scan of one value per thread over threads 0..255 of a block
// (the others pass 0 and get 0); every thread of the block must call it.
__device__ __forceinline__ uint32_t scan256(uint32_t v, uint32_t *wsum) {
  const int w = threadIdx.x >> 6;
  uint32_t ex = 0;
  if (threadIdx.x < 256) {
    int tot;
    ex = (uint32_t)wave_excl_scan_int((int)v, &tot);
    if ((threadIdx.x & 63) == 0) wsum[w] = (uint32_t)tot;
  }
  __syncthreads();
  if (threadIdx.x < 256)
    for (int ww = 0; ww < w; ++ww) ex += wsum[ww];
  __syncthreads();
  return ex;
}

// One radix pass over a tile of SORT_TILE keys: every key's rank among the
// tile's keys of its digit (8 ballots per 64 keys, waves in index order, so
// the pass is stable), the tile reordered by digit in LDS, then written out
// in tile order so that consecutive threads store consecutive addresses of a
// digit's run.
// raw = 1 (at most SORT_RAW_TILES tiles): hist holds the tiles' raw digit
// counts and each tile sums what it needs itself (no digit-scan launch);
// raw = 0: hist holds each digit's exclusive prefix over the tiles and dtot
// the digit totals.
// hist_next (raw passes but the last, else NULL): the next pass's raw counts,
// zero on entry, are accumulated here (digit next_shift / next_by_req of each
// element, by the tile of its destination), so that pass needs no histogram
// launch of its own; counts do not depend on the order they are added in.
__global__ __launch_bounds__(SORT_THREADS) void k_sort_scatter(
    const uint64_t *__restrict__ kin, const int32_t *__restrict__ sin, uint64_t *__restrict__ kout,
    int32_t *__restrict__ sout, const int32_t *__restrict__ slot_req, int n, int shift, int by_req,
    const uint32_t *__restrict__ hist, int nblk, const uint32_t *__restrict__ dtot, int raw,
    uint32_t *__restrict__ hist_next, int next_shift, int next_by_req) {
  // keys | slots | digits of the reordered tile; the per-wave digit counters
  // of the ranking step live in the front of the same space before that
  __shared__ __align__(16) unsigned char smem[SORT_TILE * 13];
  __shared__ uint32_t lstart[256], gbase[256], wsum[SORT_WAVES];
  __shared__ uint32_t lnext[256 * SORT_RAW_TILES];  // next pass's counts, [digit][tile]
  uint64_t *skey = (uint64_t *)smem;
  int32_t *sslot = (int32_t *)(smem + 8 * SORT_TILE);
  uint8_t *sdig = smem + 12 * SORT_TILE;
  uint32_t(*cnt)[256] = (uint32_t(*)[256])smem;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  for (int d = tid; d < SORT_WAVES * 256; d += SORT_THREADS) (&cnt[0][0])[d] = 0;
  // global start of each digit: exclusive scan of the digit totals, plus the
  // counts of the earlier tiles
  uint32_t dtotal = 0, tprefix = 0;
  if (tid < 256) {
    if (raw) {
      for (int b = 0; b < nblk; ++b) {
        const uint32_t c = hist[tid * nblk + b];
        dtotal += c;
        tprefix += b < (int)blockIdx.x ? c : 0u;
      }
    } else {
      dtotal = dtot[tid];
      tprefix = hist[tid * nblk + blockIdx.x];
    }
  }
  const uint32_t dbase = scan256(dtotal, wsum);
  const int tile = blockIdx.x * SORT_TILE;
  const int base = tile + w * 64 * SORT_ITEMS;
  uint64_t k[SORT_ITEMS];
  int32_t sv[SORT_ITEMS];
  uint32_t dg[SORT_ITEMS], rank[SORT_ITEMS];
  const unsigned long long below = lanes_below_mask();
#pragma unroll
  for (int it = 0; it < SORT_ITEMS; ++it) {
    const int i = base + it * 64 + lane;
    const bool valid = i < n;
    k[it] = valid ? kin[i] : 0;
    sv[it] = valid ? sin[i] : 0;
  }
#pragma unroll
  for (int it = 0; it < SORT_ITEMS; ++it) {
    const int i = base + it * 64 + lane;
    const bool valid = i < n;
    const uint32_t d = by_req ? (valid ? ((uint32_t)slot_req[sv[it]] >> shift) & 255u : 0u)
                              : (uint32_t)(k[it] >> shift) & 255u;
    dg[it] = d;
    unsigned long long m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const unsigned long long bal = __ballot((d >> b) & 1u);
      m &= ((d >> b) & 1u) ? bal : ~bal;
    }
    const uint32_t prior = cnt[w][d];
    rank[it] = prior + (uint32_t)__popcll(m & below);
    __builtin_amdgcn_wave_barrier();
    if (valid && (m & below) == 0) cnt[w][d] = prior + (uint32_t)__popcll(m);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // per digit: offsets of the waves inside the tile (in place), tile count
  uint32_t tcount = 0;
  if (tid < 256) {
#pragma unroll
    for (int ww = 0; ww < SORT_WAVES; ++ww) {
      const uint32_t c = cnt[ww][tid];
      cnt[ww][tid] = tcount;
      tcount += c;
    }
  }
  const uint32_t ls = scan256(tcount, wsum);
  if (tid < 256) {
    lstart[tid] = ls;
    gbase[tid] = dbase + tprefix - ls;
  }
  __syncthreads();
  int lpos[SORT_ITEMS];
#pragma unroll
  for (int it = 0; it < SORT_ITEMS; ++it) lpos[it] = (int)(lstart[dg[it]] + cnt[w][dg[it]] + rank[it]);
  __syncthreads();  // the counters are overwritten below
#pragma unroll
  for (int it = 0; it < SORT_ITEMS; ++it) {
    if (base + it * 64 + lane < n) {
      skey[lpos[it]] = k[it];
      sslot[lpos[it]] = sv[it];
      sdig[lpos[it]] = (uint8_t)dg[it];
    }
  }
  __syncthreads();
  const int tn = min(SORT_TILE, n - tile);
  const bool count_next = hist_next != nullptr && nblk <= SORT_RAW_TILES;
  if (count_next)
    for (int d = tid; d < 256 * nblk; d += SORT_THREADS) lnext[d] = 0;
  __syncthreads();
#pragma unroll
  for (int it = 0; it < SORT_ITEMS; ++it) {
    const int j = it * SORT_THREADS + tid;
    if (j < tn) {
      const uint32_t dst = gbase[sdig[j]] + (uint32_t)j;
      kout[dst] = skey[j];
      sout[dst] = sslot[j];
      if (count_next) {
        const uint32_t d = next_by_req ? ((uint32_t)slot_req[sslot[j]] >> next_shift) & 255u
                                       : (uint32_t)(skey[j] >> next_shift) & 255u;
        atomicAdd(&lnext[d * nblk + dst / SORT_TILE], 1u);
      }
    }
  }
  if (count_next) {
    __syncthreads();
    for (int d = tid; d < 256 * nblk; d += SORT_THREADS)
      if (lnext[d]) atomicAdd(&hist_next[d], lnext[d]);
  }
}

// Deepest level at which a cell holds more than leaf_size particles: a cell
// holds more than leaf_size particles exactly when some sorted key and the key
// leaf_size positions later (same request) share its prefix.  Cells below that
// level are leaves, so the split stops there.
__global__ __launch_bounds__(FMM_BLOCK) void k_split_depth(DevTree t, int n, int stride) {
  int best = 0;
  const uint64_t *key = t.key;
  Header *hdr = t.hdr;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i + stride < n;
       i += gridDim.x * blockDim.x) {
    if (t.n_req > 1) {  // sorted positions are grouped by request, in request order
      const int r = upper_index(t.req_off, t.n_req, i);
      if (i + stride >= t.req_off[r + 1]) continue;
    }
    uint64_t x = key[i] ^ key[i + stride];
    int digits = x == 0 ? FMM_MAXLEVEL : (__clzll(x) - 1) / 3;
    best = max(best, digits);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) best = max(best, __shfl_xor(best, off, 64));
  __shared__ int wbest[FMM_BLOCK / 64];
  if ((threadIdx.x & 63) == 0) wbest[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {  // one atomic per block
    for (int w = 1; w < FMM_BLOCK / 64; ++w) best = max(best, wbest[w]);
    if (best > 0) atomicMax(&hdr->max_prefix, best);
  }
}

// ---------------------------------------------------------------------------
// sorted particle data
// ---------------------------------------------------------------------------
// The key pass left each active slot's position in one 32-byte record, so
// the random read of the gather touches one memory sector per particle
// instead of one in each of the three coordinate arrays.
__device__ __forceinline__ void gather_at(const DevTree &t, int j) {
  const double4 r = t.pak[t.slot[j]];
  t.sx[j] = r.x;
  t.sy[j] = r.y;
  t.sz[j] = r.z;
}

__global__ __launch_bounds__(FMM_BLOCK) void k_gather_sorted(DevTree t, int n) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) gather_at(t, j);
}

// ---------------------------------------------------------------------------
// level-by-level split
// ---------------------------------------------------------------------------
__device__ __forceinline__ double4 cell_geometry(const Box &b, uint64_t prefix, int lev) {
  uint32_t ix = compact3(prefix >> 2), iy = compact3(prefix >> 1), iz = compact3(prefix);
  double w = ldexp(b.L, -lev);
  double4 g;
  g.x = b.o[0] + ((double)ix + 0.5) * w;
  g.y = b.o[1] + ((double)iy + 0.5) * w;
  g.z = b.o[2] + ((double)iz + 0.5) * w;
  g.w = ldexp(b.L, -(lev + 1));
  return g;
}

// header of a new tree (one thread) and the root of request r, covering its
// sorted range [off, off + n)
__device__ __forceinline__ void header_init(const DevTree &t) {
  Header *h = t.hdr;
  const int R = t.n_req;
  h->lvl_start[0] = 0;
  for (int l = 1; l < FMM_NLEVELS + 2; ++l) h->lvl_start[l] = R;
  h->overflow = R > t.cap_nodes ? OVF_NODES : 0;
  h->max_prefix = 0;
}

__device__ __forceinline__ void root_init(const DevTree &t, int r, int leaf_size) {
  if (r >= t.cap_nodes) return;
  t.nbeg[r] = t.req_off[r];
  t.nend[r] = t.req_off[r + 1];
  t.nlev[r] = 0;
  t.nparent[r] = -1;
  t.nchild0[r] = -1;
  t.nnchild[r] = 0;
  t.nreq[r] = r;
  t.ngeo[r] = cell_geometry(t.box[r], 0ull, 0);
  if (t.req_off[r + 1] - t.req_off[r] <= leaf_size) atomicAdd((int *)&t.hdr->n_leaves, 1);
}

__global__ __launch_bounds__(FMM_BLOCK) void k_tree_init(DevTree t, int leaf_size) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r == 0) header_init(t);
  if (r < t.n_req) root_init(t, r, leaf_size);
}

__device__ __forceinline__ int lower_bound_digit(const uint64_t *__restrict__ key, int b, int e,
                                                 int shift, uint32_t oct) {
  while (b < e) {
    int mid = (b + e) >> 1;
    if (((uint32_t)(key[mid] >> shift) & 7u) < oct)
      b = mid + 1;
    else
      e = mid;
  }
  return b;
}

__device__ __forceinline__ void level_chunk(const Header *h, int l, int &s, int &e) {
  int ls = h->lvl_start[l], le = h->lvl_start[l + 1];
  int cnt = le - ls;
  int per = (cnt + gridDim.x - 1) / gridDim.x;
  s = ls + blockIdx.x * per;
  e = min(le, s + per);
}

// children of node i of level l: octant boundaries of its key range into
// bounds[i][0..8), the number of non-empty octants into nnchild[i]
__device__ __forceinline__ int count_node(const DevTree &t, int i, int l, int leaf_size) {
  const int shift = 3 * (FMM_MAXLEVEL - (l + 1));
  int b = t.nbeg[i], en = t.nend[i];
  int nc = 0;
  if (en - b > leaf_size && l < FMM_MAXLEVEL) {
    int bd[9];
    bd[0] = b;
    bd[8] = en;
    for (uint32_t o = 1; o < 8; ++o) bd[o] = lower_bound_digit(t.key, bd[o - 1], en, shift, o);
    for (int o = 0; o < 8; ++o) {
      t.bounds[(int64_t)i * 8 + o] = bd[o];
      nc += bd[o + 1] > bd[o];
    }
  }
  t.nnchild[i] = nc;
  return nc;
}

// emit the nc children of node i (level l) at ids first, first+1, ...;
// returns how many of them are leaves
__device__ __forceinline__ int emit_node(const DevTree &t, int i, int l, int nc, int first,
                                         int leaf_size) {
  if (nc == 0) {
    t.nchild0[i] = -1;
    return 0;
  }
  int leaves = 0;
  t.nchild0[i] = first;
  const int rq = t.nreq[i];
  const Box box = t.box[rq];
  int c = first;
  for (int o = 0; o < 8; ++o) {
    int b = t.bounds[(int64_t)i * 8 + o];
    int en = o < 7 ? t.bounds[(int64_t)i * 8 + o + 1] : t.nend[i];
    if (en > b) {
      if (c < t.cap_nodes) {
        t.nbeg[c] = b;
        t.nend[c] = en;
        t.nlev[c] = l + 1;
        t.nparent[c] = i;
        t.nchild0[c] = -1;
        t.nnchild[c] = 0;
        t.nreq[c] = rq;
        uint64_t prefix = t.key[b] >> (3 * (FMM_MAXLEVEL - (l + 1)));
        t.ngeo[c] = cell_geometry(box, prefix, l + 1);
      }
      leaves += (en - b <= leaf_size || l + 1 == FMM_MAXLEVEL);
      ++c;
    }
  }
  return leaves;
}

// count_node with its searches spread over an aligned group of 8 lanes: lane
// o finds the first particle of octant >= o in the whole key range of the
// cell (its keys are sorted by octant, so this is the bound the sequential
// search finds), and the group counts the non-empty octants.  Same bounds
// and count as count_node.
__device__ __forceinline__ int count_node8(const DevTree &t, int i, int l, int leaf_size, int o) {
  const int shift = 3 * (FMM_MAXLEVEL - (l + 1));
  const int b = t.nbeg[i], en = t.nend[i];
  int nc = 0;
  if (en - b > leaf_size && l < FMM_MAXLEVEL) {
    const int bd = o == 0 ? b : lower_bound_digit(t.key, b, en, shift, (uint32_t)o);
    t.bounds[(int64_t)i * 8 + o] = bd;
    const int nx = __shfl_down(bd, 1, 8);  // lane o + 1's bound (o = 7: its own)
    const bool nonempty = o < 7 ? nx > bd : en > bd;
    const unsigned long long m = __ballot(nonempty);
    nc = __popcll((m >> (__lane_id() & 56)) & 0xFFull);
  }
  if (o == 0) t.nnchild[i] = nc;
  return nc;
}

__global__ __launch_bounds__(FMM_BLOCK) void k_tree_count(DevTree t, int l, int leaf_size) {
  int s, e;
  level_chunk(t.hdr, l, s, e);
  const int o = threadIdx.x & 7;
  int sum = 0;
  for (int i = s + (threadIdx.x >> 3); i < e && i < t.cap_nodes; i += blockDim.x >> 3) {
    const int nc = count_node8(t, i, l, leaf_size, o);
    if (o == 0) sum += nc;
  }
  __shared__ int red[FMM_BLOCK];
  red[threadIdx.x] = sum;
  __syncthreads();
  for (int o = FMM_BLOCK / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) t.scan_part[blockIdx.x] = red[0];
}


// Children of the splitting cells of level l; a child is a leaf when it holds
// at most leaf_size particles or sits at the deepest level, and leaves are
// counted here.
// Sum of v over a block of FMM_BLOCK threads (all of them call it).
__device__ __forceinline__ int block_sum(int v, int *part) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  int tot = 0;
#pragma unroll
  for (int w = 0; w < FMM_BLOCK / 64; ++w) tot += part[w];
  __syncthreads();
  return tot;
}

// Each block first takes its offset among the children of the level (the
// child counts of the earlier blocks, from k_tree_count) and the level's
// total; block 0 records where the next level ends.
__global__ __launch_bounds__(FMM_BLOCK) void k_tree_emit(DevTree t, int l, int leaf_size) {
  static_assert(FMM_SCAN_BLOCKS == FMM_BLOCK, "one block count per thread");
  int s, e;
  level_chunk(t.hdr, l, s, e);
  __shared__ int sc[FMM_BLOCK];
  __shared__ int part[FMM_BLOCK / 64];
  const int cnt = t.scan_part[threadIdx.x];
  const int before = block_sum((int)threadIdx.x < (int)blockIdx.x ? cnt : 0, part);
  const int level_total = block_sum(cnt, part);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Header *h = t.hdr;
    const int next = h->lvl_start[l + 1] + level_total;
    for (int k = l + 2; k < FMM_NLEVELS + 2; ++k) h->lvl_start[k] = next;
    if (next > t.cap_nodes) h->overflow |= OVF_NODES;
  }
  int run = t.hdr->lvl_start[l + 1] + before;
  for (int base = s; base < e; base += FMM_BLOCK) {
    int i = base + threadIdx.x;
    int nc = (i < e && i < t.cap_nodes) ? t.nnchild[i] : 0;
    sc[threadIdx.x] = nc;
    __syncthreads();
    for (int off = 1; off < FMM_BLOCK; off <<= 1) {
      int y = threadIdx.x >= off ? sc[threadIdx.x - off] : 0;
      __syncthreads();
      sc[threadIdx.x] += y;
      __syncthreads();
    }
    int first = run + sc[threadIdx.x] - nc;
    int total = sc[FMM_BLOCK - 1];
    __syncthreads();
    int leaves = 0;
    if (i < e && i < t.cap_nodes) leaves = emit_node(t, i, l, nc, first, leaf_size);
    if (leaves) atomicAdd((int *)&t.hdr->n_leaves, leaves);
    run += total;
  }
}

// ---------------------------------------------------------------------------
// Every split level at once (leaf_size <= TD_MAXLEAF): a fixed number of
// launches whatever the depth, and no host read of the split depth first.
//
// The cell of level l that holds sorted particle i (a run of keys sharing
// their first l octal digits) holds more than L = leaf_size particles exactly
// when some k in [i - L, i] of the same system has keys k and k + L sharing
// those digits (then k .. k + L, which contains i, lies in the run; and a run
// of more than L particles contains such a window around any of its
// particles).  With c(k) the common leading levels of keys k and k + L, the
// cells along i's path are split at levels 0 .. m, m the largest c(k) over
// that window, and i's leaf is at level d(i) = m + 1 (0 when no window fits
// in the system; at most FMM_MAXLEVEL).  A cell of level l >= 1 exists when
// its parent is split, i.e. l <= d(i) for its particles, and particle i
// starts one at every level l from cp(i) + 1 to d(i), cp(i) the common
// levels of keys i - 1 and i (0 at the first particle of a system); it ends
// the run of every level l from cp(i + 1) + 1 (0 at the system's last
// particle) to d(i).  Nodes are numbered level by level, in sorted order
// within a level, as the level-by-level split numbers them, so the two build
// the same tree bit for bit.
// ---------------------------------------------------------------------------
#define TD_THREADS 1024
#define TD_WAVES (TD_THREADS / 64)
#define TD_MAXLEAF 1024

__device__ __forceinline__ int common_levels(uint64_t a, uint64_t b) {
  const uint64_t x = a ^ b;
  return x == 0 ? FMM_MAXLEVEL : (__clzll(x) - 1) / 3;
}

// c(i) into slot2 (free after the sort): -1 when i + L is past the system
__global__ __launch_bounds__(FMM_BLOCK) void k_tree_pairs(DevTree t, int n, int L) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int r = t.n_req > 1 ? upper_index(t.req_off, t.n_req, i) : 0;
  t.slot2[i] = i + L < t.req_off[r + 1] ? common_levels(t.key[i], t.key[i + L]) : -1;
}

// per-particle level data, packed: d | lo << 8 | lo2 << 16 (lo: first level
// >= 1 at which i starts a cell; lo2: first level at which i ends a run)
__device__ __forceinline__ void td_unpack(uint64_t v, int &d, int &lo, int &lo2) {
  d = (int)(v & 255u);
  lo = (int)((v >> 8) & 255u);
  lo2 = (int)((v >> 16) & 255u);
}

// d, lo, lo2 of every particle into key2, and per level l >= 1 the number of
// cells of level l that start in each block of TD_THREADS particles into
// hist[(l - 1) * nblk + block]
__global__ __launch_bounds__(TD_THREADS) void k_tree_levels(DevTree t, int n, int L, int nblk,
                                                            uint32_t *hist) {
  __shared__ int cw[TD_THREADS + TD_MAXLEAF];  // c over [b0 - L, b0 + TD_THREADS)
  __shared__ int wcnt[TD_WAVES][FMM_MAXLEVEL];
  const int b0 = blockIdx.x * TD_THREADS;
  for (int k = threadIdx.x; k < TD_THREADS + L; k += TD_THREADS) {
    const int g = b0 - L + k;
    cw[k] = (g >= 0 && g < n) ? t.slot2[g] : -1;
  }
  __syncthreads();
  const int i = b0 + threadIdx.x;
  int lo = 1, hi = 0;
  if (i < n) {
    const int r = t.n_req > 1 ? upper_index(t.req_off, t.n_req, i) : 0;
    const int rs = t.req_off[r], re = t.req_off[r + 1];
    int m = -1;
    for (int k = max(i - L, rs); k <= i; ++k) m = max(m, cw[k - b0 + L]);
    const int d = m < 0 ? 0 : min(FMM_MAXLEVEL, m + 1);
    const int cpi = i == rs ? 0 : common_levels(t.key[i - 1], t.key[i]);
    const int lo2 = i + 1 == re ? 0 : common_levels(t.key[i], t.key[i + 1]) + 1;
    lo = cpi + 1;
    hi = d;
    t.key2[i] = (uint64_t)d | ((uint64_t)lo << 8) | ((uint64_t)lo2 << 16);
  }
  const int w = threadIdx.x >> 6;
  for (int l = 1; l <= FMM_MAXLEVEL; ++l) {
    const unsigned long long b = __ballot(lo <= l && l <= hi);
    if ((threadIdx.x & 63) == 0) wcnt[w][l - 1] = __popcll(b);
  }
  __syncthreads();
  if (threadIdx.x < FMM_MAXLEVEL) {
    int s = 0;
    for (int ww = 0; ww < TD_WAVES; ++ww) s += wcnt[ww][threadIdx.x];
    hist[(size_t)threadIdx.x * nblk + blockIdx.x] = (uint32_t)s;
  }
}

// The nodes of levels >= 1 and the children of the roots.  hist holds, per
// level, each block's exclusive offset among the level's cells, tot the
// level totals.  A split cell's child count is written first as the end of
// its children (by the particle that ends the cell) and turned into a count
// by k_tree_nchild.
__global__ __launch_bounds__(TD_THREADS) void k_tree_nodes(DevTree t, int n, int nblk,
                                                           const uint32_t *hist,
                                                           const uint32_t *tot, int walk_levels) {
  __shared__ int wpre[TD_WAVES][FMM_MAXLEVEL];
  __shared__ int lvs_s[FMM_NLEVELS + 2];
  __shared__ int leaves_w[TD_WAVES];
  if (threadIdx.x == 0) {
    lvs_s[0] = 0;
    lvs_s[1] = t.n_req;
    for (int l = 1; l <= FMM_NLEVELS; ++l)
      lvs_s[l + 1] = lvs_s[l] + (l <= FMM_MAXLEVEL ? (int)tot[l - 1] : 0);
  }
  const int b0 = blockIdx.x * TD_THREADS;
  const int i = b0 + threadIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int d = 0, lo = 1, lo2 = FMM_MAXLEVEL + 1, r = 0;
  if (i < n) {
    td_unpack(t.key2[i], d, lo, lo2);
    r = t.n_req > 1 ? upper_index(t.req_off, t.n_req, i) : 0;
  }
  const int hi = i < n ? d : 0;
  const unsigned long long below = lanes_below_mask();
  int rank[FMM_MAXLEVEL + 2];  // exclusive rank among the level's cell starts, levels 1..
  for (int l = 1; l <= FMM_MAXLEVEL; ++l) {
    const unsigned long long b = __ballot(lo <= l && l <= hi);
    rank[l] = __popcll(b & below);
    if (lane == 0) wpre[w][l - 1] = __popcll(b);
  }
  rank[0] = rank[FMM_MAXLEVEL + 1] = 0;
  __syncthreads();
  if (threadIdx.x < FMM_MAXLEVEL) {  // exclusive prefix over the waves, in place
    int run = 0;
    for (int ww = 0; ww < TD_WAVES; ++ww) {
      const int c = wpre[ww][threadIdx.x];
      wpre[ww][threadIdx.x] = run;
      run += c;
    }
  }
  __syncthreads();
  for (int l = 1; l <= FMM_MAXLEVEL; ++l)
    rank[l] += wpre[w][l - 1] + (int)hist[(size_t)(l - 1) * nblk + blockIdx.x];
  const int64_t cap = t.cap_nodes;
  int leaves = 0;
  if (i < n) {
    const Box box = t.box[r];
    // cells that start at i
    for (int l = lo; l <= hi; ++l) {
      const int64_t k = (int64_t)lvs_s[l] + rank[l];
      const bool split = l < d;
      leaves += !split;
      if (k >= cap) continue;
      const bool ps = lo <= l - 1;  // i also starts its parent
      t.nbeg[k] = i;
      t.nlev[k] = l;
      t.nparent[k] = l == 1 ? r : lvs_s[l - 1] + rank[l - 1] + (ps ? 1 : 0) - 1;
      t.nchild0[k] = split ? lvs_s[l + 1] + rank[l + 1] : -1;
      if (!split) t.nnchild[k] = 0;
      t.nreq[k] = r;
      t.ngeo[k] = cell_geometry(box, t.key[i] >> (3 * (FMM_MAXLEVEL - l)), l);
    }
    // the root's children start at the system's first particle
    if (lo == 1 && i == t.req_off[r] && d > 0 && r < cap) t.nchild0[r] = lvs_s[1] + rank[1];
    // runs that end at i
    for (int l = lo2; l <= hi; ++l) {
      const bool split = l < d;
      const int incl_next = split ? rank[l + 1] + (lo <= l + 1 ? 1 : 0) : 0;
      if (l == 0) {
        if (split && r < cap) t.nnchild[r] = lvs_s[1] + incl_next;
        continue;
      }
      const int64_t k = (int64_t)lvs_s[l] + rank[l] + (lo <= l ? 1 : 0) - 1;
      if (k >= cap) continue;
      t.nend[k] = i + 1;
      if (split) t.nnchild[k] = lvs_s[l + 1] + incl_next;
    }
  }
  leaves = wave_sum(leaves);
  if (lane == 0) leaves_w[w] = leaves;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int ww = 0; ww < TD_WAVES; ++ww) s += leaves_w[ww];
    if (s) atomicAdd((int *)&t.hdr->n_leaves, s);
    if (blockIdx.x == 0) {
      Header *h = t.hdr;
      for (int l = 0; l < FMM_NLEVELS + 2; ++l) h->lvl_start[l] = lvs_s[l];
      if (lvs_s[FMM_NLEVELS + 1] > cap) h->overflow |= OVF_NODES;
      int deepest = 0;
      for (int l = 1; l <= FMM_MAXLEVEL; ++l)
        if (lvs_s[l + 1] > lvs_s[l]) deepest = l;
      if (deepest > walk_levels) h->overflow |= OVF_DEPTH;
    }
  }
}

// split cells: child count = end of the children - first child
__global__ __launch_bounds__(FMM_BLOCK) void k_tree_nchild(DevTree t) {
  const int total = min(t.hdr->lvl_start[FMM_NLEVELS + 1], (int)t.cap_nodes);
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < total; k += gridDim.x * blockDim.x) {
    const int c0 = t.nchild0[k];
    if (c0 >= 0) t.nnchild[k] -= c0;
  }
}

// ---------------------------------------------------------------------------
// Small batches (at most SMALL_N active particles in all): the whole build up
// to the walk -- slots, boxes, roots, keys, every sort pass, sorted gather,
// split depth and every split level -- in one workgroup, one launch, with no
// host round trip.  Each step is the same per-element code as the multi-block
// path, so the tree is the same bit for bit.
// ---------------------------------------------------------------------------
// block-wide exclusive scan of one int per thread (wave shuffles, then the
// wave totals through LDS); *total gets the sum
__device__ __forceinline__ int block_excl_scan_small(int v, int *wsum, int *total) {
  const int w = threadIdx.x >> 6;
  int wt;
  const int x = wave_excl_scan_int(v, &wt);
  if ((threadIdx.x & 63) == 0) wsum[w] = wt;
  __syncthreads();
  int off = 0, tot = 0;
  for (int k = 0; k < SMALL_WAVES; ++k) {
    off += k < w ? wsum[k] : 0;
    tot += wsum[k];
  }
  __syncthreads();
  *total = tot;
  return off + x;
}

__global__ __launch_bounds__(SMALL_THREADS) void k_build_small(DevTree t, int n, int leaf_size,
                                                               int req_passes) {
  __shared__ uint32_t cnt[SMALL_WAVES][256];
  __shared__ uint32_t dbase[256];
  __shared__ uint64_t skey[SMALL_THREADS];
  __shared__ int sord[SMALL_THREADS];
  __shared__ int wsum[SMALL_WAVES];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int T = SMALL_THREADS;
  Header *h = t.hdr;
  if (tid == 0) {
    h->nonfinite = 0;
    h->n_leaves = 0;
    header_init(t);
  }
  for (int q = tid; q < n; q += T) t.slot_req[q] = upper_index(t.req_off, t.n_req, q);
  // root box of every request: one wavefront per request
  int bad = 0;
  for (int r = w; r < t.n_req; r += SMALL_WAVES) {
    const DevReq q = t.reqs[r];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = lane; i < q.n; i += 64) {
      int64_t g = q.active ? q.active[i] : i;
      for (int d = 0; d < 3; ++d) {
        double x = q.pos[d * q.n_total + g];
        bad |= !isfinite(x);
        lo[d] = fmin(lo[d], x);
        hi[d] = fmax(hi[d], x);
      }
    }
    for (int off = 32; off > 0; off >>= 1)
      for (int d = 0; d < 3; ++d) {
        lo[d] = fmin(lo[d], __shfl_xor(lo[d], off, 64));
        hi[d] = fmax(hi[d], __shfl_xor(hi[d], off, 64));
      }
    if (lane == 0) finish_box(t.box[r], lo, hi, q.n == 0);
  }
  if (__syncthreads_or(bad) && tid == 0) h->nonfinite = 1;
  for (int r = tid; r < t.n_req; r += T) root_init(t, r, leaf_size);
  for (int q = tid; q < n; q += T) make_key(t, q, t.key, t.slot);
  __syncthreads();
  if (n <= T) {
    // at most one particle per thread: the rank of (request, key, slot) among
    // all of them is its place in the stable sorted order
    uint64_t k = 0;
    int r = 0;
    if (tid < n) {
      k = t.key[tid];
      r = t.slot_req[tid];
      skey[tid] = k;
      sord[tid] = r;
    }
    __syncthreads();
    if (tid < n) {
      int rank = 0;
      for (int j = 0; j < n; ++j) {
        const int rj = sord[j];
        const uint64_t kj = skey[j];
        rank += (rj < r) || (rj == r && (kj < k || (kj == k && j < tid)));
      }
      t.key[rank] = k;
      t.slot[rank] = tid;  // slots are still in input order
    }
    __syncthreads();
  } else {
    // stable LSD radix sort, 8-bit digits: 8 key passes, then request passes
    uint64_t *kin = t.key, *kout = t.key2;
    int32_t *sin = t.slot, *sout = t.slot2;
    const unsigned long long below = lanes_below_mask();
    const int base = w * 64 * SMALL_ITEMS;
    const int items = min(SMALL_ITEMS, max(0, (n - base + 63) / 64));  // uniform per wave
    for (int pass = 0; pass < 8 + req_passes; ++pass) {
      const int by_req = pass >= 8;
      const int shift = by_req ? (pass - 8) * 8 : pass * 8;
      for (int d = tid; d < SMALL_WAVES * 256; d += T) (&cnt[0][0])[d] = 0;
      __syncthreads();
      uint64_t k[SMALL_ITEMS];
      int32_t sv[SMALL_ITEMS];
      uint32_t rank[SMALL_ITEMS], dg[SMALL_ITEMS];
#pragma unroll
      for (int it = 0; it < SMALL_ITEMS; ++it) {
        if (it >= items) continue;  // wave-uniform
        int i = base + it * 64 + lane;
        bool valid = i < n;
        k[it] = valid ? kin[i] : 0;
        sv[it] = valid ? sin[i] : 0;
        uint32_t d = by_req ? ((uint32_t)t.slot_req[sv[it]] >> shift) & 255u
                            : (uint32_t)(k[it] >> shift) & 255u;
        dg[it] = d;
        unsigned long long m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          unsigned long long bal = __ballot((d >> b) & 1u);
          m &= ((d >> b) & 1u) ? bal : ~bal;
        }
        uint32_t prior = cnt[w][d];
        rank[it] = prior + (uint32_t)__popcll(m & below);
        __builtin_amdgcn_wave_barrier();
        if (valid && (m & below) == 0) cnt[w][d] = prior + (uint32_t)__popcll(m);
        __builtin_amdgcn_wave_barrier();
      }
      __syncthreads();
      if (w == 0) {  // digit bases: lane l scans digits 4l .. 4l+3
        uint32_t tt[4], sum = 0;
        for (int q = 0; q < 4; ++q) {
          tt[q] = 0;
          for (int ww = 0; ww < SMALL_WAVES; ++ww) tt[q] += cnt[ww][4 * lane + q];
          sum += tt[q];
        }
        int tot;
        uint32_t run = (uint32_t)wave_excl_scan_int((int)sum, &tot);
        for (int q = 0; q < 4; ++q) {
          dbase[4 * lane + q] = run;
          run += tt[q];
        }
      }
      __syncthreads();
      if (tid < 256) {
        uint32_t run = dbase[tid];
        for (int ww = 0; ww < SMALL_WAVES; ++ww) {
          const uint32_t c = cnt[ww][tid];
          cnt[ww][tid] = run;
          run += c;
        }
      }
      __syncthreads();
#pragma unroll
      for (int it = 0; it < SMALL_ITEMS; ++it) {
        int i = base + it * 64 + lane;
        if (it < items && i < n) {
          uint32_t dst = cnt[w][dg[it]] + rank[it];
          kout[dst] = k[it];
          sout[dst] = sv[it];
        }
      }
      __syncthreads();
      uint64_t *tk = kin; kin = kout; kout = tk;
      int32_t *ts = sin; sin = sout; sout = ts;
    }
  }
  // sorted positions; split depth (keys leaf_size apart, same request)
  int best = 0;
  for (int i = tid; i < n; i += T) {
    gather_at(t, i);
    if (i + leaf_size < n) {
      const int r = t.n_req > 1 ? upper_index(t.req_off, t.n_req, i) : 0;
      if (t.n_req == 1 || i + leaf_size < t.req_off[r + 1]) {
        uint64_t x = t.key[i] ^ t.key[i + leaf_size];
        best = max(best, x == 0 ? FMM_MAXLEVEL : (__clzll(x) - 1) / 3);
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) best = max(best, __shfl_xor(best, off, 64));
  if (lane == 0) wsum[w] = best;
  __syncthreads();
  for (int k2 = 0; k2 < SMALL_WAVES; ++k2) best = max(best, wsum[k2]);
  if (tid == 0) h->max_prefix = best;
  const int max_level = min(FMM_MAXLEVEL, best + 1);
  __syncthreads();
  // level-by-level split
  int leaves = 0;
  int ls = 0, run = t.n_req;  // level l occupies [ls, run) when its split starts
  for (int l = 0; l < max_level; ++l) {
    const int le = min(run, (int)t.cap_nodes);
    int next = run;
    for (int b0 = ls; b0 < le; b0 += T) {
      const int i = b0 + tid;
      const int nc = i < le ? count_node(t, i, l, leaf_size) : 0;
      int total;
      const int first = next + block_excl_scan_small(nc, wsum, &total);
      if (i < le) leaves += emit_node(t, i, l, nc, first, leaf_size);
      next += total;
    }
    if (tid == 0) {
      for (int k2 = l + 2; k2 < FMM_NLEVELS + 2; ++k2) h->lvl_start[k2] = next;
      if (next > t.cap_nodes) h->overflow |= OVF_NODES;
    }
    ls = run;
    run = next;
    __syncthreads();
  }
  int total;
  block_excl_scan_small(leaves, wsum, &total);
  if (tid == 0 && total) atomicAdd((int *)&h->n_leaves, total);
}

hipError_t launch_build_small(const DevTree &t, const BuildArgs &a, hipStream_t s) {
  if (a.tm) a.tm->start(PH_TREE, s);
  const int req_passes = a.n_req > 1 ? (a.n_req > 65536 ? 4 : 2) : 0;
  hipLaunchKernelGGL(k_build_small, dim3(1), dim3(SMALL_THREADS), 0, s, t, a.n, a.leaf_size,
                     req_passes);
  if (a.tm) a.tm->stop(s);
  return hipGetLastError();
}

hipError_t launch_sort(const DevTree &t, const BuildArgs &a, hipStream_t s) {
  const int n = a.n;
  const int nb = (n + FMM_BLOCK - 1) / FMM_BLOCK;
  if (a.tm) a.tm->start(PH_SORT, s);
  hipLaunchKernelGGL(k_slot_req, dim3(std::max(nb, 1)), dim3(FMM_BLOCK), 0, s, t, n);
  hipLaunchKernelGGL(k_bbox_partial, dim3(a.n_blk), dim3(FMM_BLOCK), 0, s, t);
  hipLaunchKernelGGL(k_bbox_final, dim3((a.n_req + 3) / 4), dim3(FMM_BLOCK), 0, s, t);
  hipLaunchKernelGGL(k_tree_init, dim3((a.n_req + FMM_BLOCK - 1) / FMM_BLOCK), dim3(FMM_BLOCK), 0,
                     s, t, a.leaf_size);
  if (n > 0) {
    const int nblk = (n + SORT_TILE - 1) / SORT_TILE;
    // 8 passes over the 63-bit key, then (several requests) one pass per byte
    // of the largest request id; with an odd number of passes the keys start
    // in key2 / slot2, so that the result always lands in key / slot
    int req_passes = 0;
    if (a.n_req > 1) req_passes = a.n_req > 65536 ? 4 : (a.n_req > 256 ? 2 : 1);
    const int passes = 8 + req_passes;
    const int odd = passes & 1;
    hipLaunchKernelGGL(k_keys, dim3(nb), dim3(FMM_BLOCK), 0, s, t, n, odd);
    uint64_t *kin = odd ? t.key2 : t.key, *kout = odd ? t.key : t.key2;
    int32_t *sin = odd ? t.slot2 : t.slot, *sout = odd ? t.slot : t.slot2;
    const int raw = nblk <= SORT_RAW_TILES;
    // raw passes: one histogram slice per pass, the first counted by
    // k_sort_hist (which clears the others), each later one by the scatter
    // before it
    const int slice = 256 * nblk;
    for (int pass = 0; pass < passes; ++pass) {
      const int by_req = pass >= 8;
      const int shift = by_req ? (pass - 8) * 8 : pass * 8;
      const int nx = pass + 1;
      const int next_by_req = nx >= 8;
      const int next_shift = next_by_req ? (nx - 8) * 8 : nx * 8;
      uint32_t *hist = raw ? t.sort_hist + (size_t)pass * slice : t.sort_hist;
      uint32_t *hist_next = raw && nx < passes ? t.sort_hist + (size_t)nx * slice : nullptr;
      if (!raw || pass == 0)
        hipLaunchKernelGGL(k_sort_hist, dim3(nblk), dim3(SORT_THREADS), 0, s, kin, sin, t.slot_req,
                           n, shift, by_req, hist, nblk, raw ? passes - 1 : 0);
      if (!raw)
        hipLaunchKernelGGL(k_sort_digit_scan, dim3(256), dim3(FMM_BLOCK), 0, s, t.sort_hist, nblk,
                           t.sort_dtot);
      hipLaunchKernelGGL(k_sort_scatter, dim3(nblk), dim3(SORT_THREADS), 0, s, kin, sin, kout, sout,
                         t.slot_req, n, shift, by_req, hist, nblk, t.sort_dtot, raw, hist_next,
                         next_shift, next_by_req);
      uint64_t *tk = kin; kin = kout; kout = tk;
      int32_t *ts = sin; sin = sout; sout = ts;
    }
    hipLaunchKernelGGL(k_gather_sorted, dim3(nb), dim3(FMM_BLOCK), 0, s, t, n);
    hipLaunchKernelGGL(k_split_depth, dim3(std::min(nb, 512)), dim3(FMM_BLOCK), 0, s, t, n,
                       a.leaf_size);
  }
  if (a.tm) a.tm->stop(s);
  return hipGetLastError();
}

// Every level at once (see k_tree_levels); false when leaf_size is beyond the
// window that fits in LDS (then launch_build_tree builds level by level).
bool build_tree_direct_ok(int leaf_size) { return leaf_size >= 1 && leaf_size <= TD_MAXLEAF; }

// walk_levels: the levels the walk that follows covers (a deeper tree is
// flagged with OVF_DEPTH and not evaluated)
hipError_t launch_build_tree_direct(const DevTree &t, const BuildArgs &a, int walk_levels,
                                    hipStream_t s) {
  const int n = a.n;
  if (a.tm) a.tm->start(PH_TREE, s);
  if (n > 0) {
    const int L = a.leaf_size;
    const int nblk = (n + TD_THREADS - 1) / TD_THREADS;
    hipLaunchKernelGGL(k_tree_pairs, dim3((n + FMM_BLOCK - 1) / FMM_BLOCK), dim3(FMM_BLOCK), 0, s,
                       t, n, L);
    hipLaunchKernelGGL(k_tree_levels, dim3(nblk), dim3(TD_THREADS), 0, s, t, n, L, nblk,
                       t.sort_hist);
    hipLaunchKernelGGL(k_sort_digit_scan, dim3(FMM_MAXLEVEL), dim3(FMM_BLOCK), 0, s, t.sort_hist,
                       nblk, t.sort_dtot);
    hipLaunchKernelGGL(k_tree_nodes, dim3(nblk), dim3(TD_THREADS), 0, s, t, n, nblk, t.sort_hist,
                       t.sort_dtot, walk_levels);
    hipLaunchKernelGGL(k_tree_nchild, dim3(std::min(1024, std::max(1, n / 256))), dim3(FMM_BLOCK),
                       0, s, t);
  }
  if (a.tm) a.tm->stop(s);
  return hipGetLastError();
}

// levels 0 .. max_level-1 are split (cells of level max_level are leaves)
hipError_t launch_build_tree(const DevTree &t, const BuildArgs &a, int max_level, hipStream_t s) {
  const int n = a.n;
  if (a.tm) a.tm->start(PH_TREE, s);
  if (n > 0) {
    for (int l = 0; l < max_level && l < FMM_MAXLEVEL; ++l) {
      hipLaunchKernelGGL(k_tree_count, dim3(FMM_SCAN_BLOCKS), dim3(FMM_BLOCK), 0, s, t, l,
                         a.leaf_size);
      hipLaunchKernelGGL(k_tree_emit, dim3(FMM_SCAN_BLOCKS), dim3(FMM_BLOCK), 0, s, t, l,
                         a.leaf_size);
    }
  }
  if (a.tm) a.tm->stop(s);
  return hipGetLastError();
}


