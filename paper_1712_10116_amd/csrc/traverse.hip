// Symmetric dual tree walk (Sec. 2.3, Algorithm 4 with "open both") on gfx950.
//
// The walk over cell pairs starting from (root, root) visits a pair (A, C)
// and then:  accepts it for M2L if it is well separated; makes it a P2P pair
// if both are leaves; opens the non-leaf cell if exactly one is a leaf; opens
// BOTH cells otherwise.  The rule is symmetric in A and C, so the set of
// visited ordered pairs is closed under swapping and every unordered
// interaction appears in both cells' lists.
//
// Target-centric form used here: a visited pair (A, C) with A not a leaf and
// not accepted is recorded in A's "open" list; the children of A then inherit
// the candidates {children of C} (or C itself if C is a leaf).  A leaf target
// that meets a non-leaf candidate descends into that candidate's children on
// a per-wavefront LDS stack.  One wavefront handles all children of one cell
// (siblings share their candidates, which are expanded once into LDS and
// tested against every sibling); level l of the tree is one launch.  Outputs
// are written in two passes (count, then write after an atomic allocation),
// so each cell's lists are contiguous and their content and order are
// deterministic.
//
// Well-separation is Eq. (1) with R = half side, plus the softening rule of
// Sec. 2.3, written in IEEE double without contraction:
//   d2 = (dx*dx + dy*dy) + dz*dz,  S = hA + hB,
//   d2*(theta*theta) > S*S  and  d2 > (eps + sqrt(3)*S)^2.
#include <algorithm>

#include "common.h"

#define TRAV_WAVES 2
#define TRAV_CAND 512   // expanded candidates of one block of 64 open-list entries
#define TRAV_STACK 768  // descent items (target tag in the top 3 bits)
// Room kept free for single-item (depth-first) pops: each pops one item and
// pushes at most its 8 children, one level deeper, so a depth-first run from
// any state grows the stack by at most 7 per level below it.
#define TRAV_RESERVE (7 * (FMM_MAXLEVEL + 1))
#define TRAV_TAG 28

enum { CAT_NONE = 0, CAT_M2L = 1, CAT_P2P = 2, CAT_OPEN = 3, CAT_DEEPEN = 4 };

__device__ __forceinline__ bool well_separated(const double4 a, const double4 b, double th2,
                                               double eps) {
  double dx = a.x - b.x;
  double dy = a.y - b.y;
  double dz = a.z - b.z;
  double d2 = (dx * dx + dy * dy) + dz * dz;
  double S = a.w + b.w;
  bool mac = d2 * th2 > S * S;
  double e = eps + 1.7320508075688772 * S;
  bool sep = d2 > e * e;
  return mac && sep;
}

__device__ __forceinline__ int classify(int A, const double4 &gA, bool leafA, int C,
                                        const double4 &gC, bool leafC, double th2, double eps) {
  if (C == A) return leafA ? CAT_P2P : CAT_OPEN;
  if (well_separated(gA, gC, th2, eps)) return CAT_M2L;
  if (leafA) return leafC ? CAT_P2P : CAT_DEEPEN;
  return CAT_OPEN;
}

// Per-wavefront state of the sibling targets (children of one parent cell).
struct Sibs {
  int n;          // number of targets, 1..8
  int id[8];
  bool leaf[8];
  int np[8];      // particles per target
  int cnt[8][3];  // M2L / P2P / OPEN entries counted (pass 0) or written (pass 1)
  int off[8][3];  // list offsets (pass 1)
};

struct WaveLds {
  int cand[TRAV_CAND];   // candidates expanded from a block of open-list entries
  int ccat[TRAV_CAND];   // their categories against the 8 targets (3 bits each), kept
                         // from the counting pass for the writing pass
  int dcand[TRAV_CAND];  // children of popped descent items
  int stack[TRAV_STACK]; // descent items: (target tag << TRAV_TAG) | cell
  double4 geo[8];
  int sid[8];            // target cells and their leaf flags, for per-lane lookup
  int sleaf[8];
};

template <bool WRITE>
__device__ __forceinline__ void emit(const DevTree &t, Sibs &S, int tg, int cat, bool mine, int C,
                                     int npC, int *open_out, unsigned long long &pairs) {
  const unsigned long long below = lanes_below_mask();
  const unsigned long long bm = __ballot(mine && cat == CAT_M2L);
  const unsigned long long bp = __ballot(mine && cat == CAT_P2P);
  const unsigned long long bo = __ballot(mine && cat == CAT_OPEN);
  if (WRITE) {
    if (mine && cat == CAT_M2L) t.m2l_src[S.off[tg][0] + S.cnt[tg][0] + __popcll(bm & below)] = C;
    if (mine && cat == CAT_P2P) t.p2p_src[S.off[tg][1] + S.cnt[tg][1] + __popcll(bp & below)] = C;
    if (mine && cat == CAT_OPEN) open_out[S.off[tg][2] + S.cnt[tg][2] + __popcll(bo & below)] = C;
  } else if (mine && cat == CAT_P2P) {  // particle pairs, counted once (counting pass)
    pairs += (unsigned long long)S.np[tg] * (unsigned long long)npC -
             (C == S.id[tg] ? (unsigned long long)S.np[tg] : 0ull);
  }
  S.cnt[tg][0] += __popcll(bm);
  S.cnt[tg][1] += __popcll(bp);
  S.cnt[tg][2] += __popcll(bo);
}

// push (tg, C) for every lane whose leaf target descends into C
__device__ __forceinline__ void push_item(const DevTree &t, WaveLds &L, int &sp, bool push, int tg,
                                          int C) {
  const unsigned long long m = __ballot(push);
  const int k = __popcll(m);
  if (sp + k > TRAV_STACK) {  // cannot happen (see drain); kept as a guard
    if (__lane_id() == 0) atomicOr(&t.hdr->overflow, OVF_STACK);
    return;
  }
  if (push) L.stack[sp + __popcll(m & lanes_below_mask())] = (tg << TRAV_TAG) | C;
  sp += k;
}

// Descents of leaf targets into non-leaf cells, LIFO.  A popped item (tg, C)
// makes the children of C candidates of target tg; each may push one item.
// Batches of take <= (TRAV_STACK - TRAV_RESERVE - sp) / 7 items keep sp below
// TRAV_STACK - TRAV_RESERVE; once that room is used up, items are popped one
// at a time (depth first), which the reserve absorbs.
template <bool WRITE>
__device__ void drain(const DevTree &t, Sibs &S, WaveLds &L, int &sp, int *open_out, double th2,
                      double eps, unsigned long long &pairs) {
  const int lane = __lane_id();
  while (sp > 0) {
    const int room = (TRAV_STACK - TRAV_RESERVE - sp) / 7;
    const int take = min(sp, max(1, min(64, room)));
    const bool vp = lane < take;
    const int item = vp ? L.stack[sp - take + lane] : 0;
    __builtin_amdgcn_wave_barrier();
    sp -= take;
    const int tgi = item >> TRAV_TAG;
    const int Ci = item & ((1 << TRAV_TAG) - 1);
    const int nCi = vp ? t.nnchild[Ci] : 0;
    const int c0 = vp ? t.nchild0[Ci] : 0;
    int total;
    const int pos = wave_excl_scan_int(nCi, &total);
    for (int q = 0; q < nCi; ++q) L.dcand[pos + q] = (tgi << TRAV_TAG) | (c0 + q);
    __builtin_amdgcn_wave_barrier();
    for (int cb = 0; cb < total; cb += 64) {
      const bool valid = cb + lane < total;
      const int it = valid ? L.dcand[cb + lane] : 0;
      const int tgl = it >> TRAV_TAG;
      const int C = it & ((1 << TRAV_TAG) - 1);
      double4 gC = make_double4(0, 0, 0, 0);
      int nC = 0, npC = 0;
      if (valid) {
        gC = t.ngeo[C];
        nC = t.nnchild[C];
        npC = t.nend[C] - t.nbeg[C];
      }
      // each lane's item belongs to one target: classify once against it
      const int lcat = valid ? classify(L.sid[tgl], L.geo[tgl], L.sleaf[tgl] != 0, C, gC,
                                        nC == 0, th2, eps)
                             : CAT_NONE;
#pragma unroll
      for (int tg = 0; tg < 8; ++tg) {
        if (tg < S.n) {
          const bool mine = valid && tgl == tg;
          if (__ballot(mine) == 0ull) continue;  // no item of this target in the chunk
          const int cat = mine ? lcat : CAT_NONE;
          emit<WRITE>(t, S, tg, cat, mine, C, npC, open_out, pairs);
          push_item(t, L, sp, cat == CAT_DEEPEN, tg, C);
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// One pass over the candidates of a sibling group (pass 0 counts, pass 1 writes).
// With at most 64 open-list entries (one block of candidates, the usual
// case) the counting pass keeps every candidate's categories in LDS and the
// writing pass replays them: it reads no cell data for these candidates (its
// only global accesses are the list stores and the descents).  ncand: the
// number of cached candidates, set by the counting pass (0 when it expanded
// none, e.g. an open list emptied by an overflow) and read by the writing pass.
template <bool WRITE>
__device__ void walk_group(const DevTree &t, int l, int P, Sibs &S, WaveLds &L,
                           const int *open_in, int *open_out, double th2, double eps,
                           unsigned long long &pairs, int &ncand) {
  const int lane = __lane_id();
#pragma unroll
  for (int tg = 0; tg < 8; ++tg) S.cnt[tg][0] = S.cnt[tg][1] = S.cnt[tg][2] = 0;
  int sp = 0;
  int in_off = 0, in_cnt = 1;
  if (l > 0) {
    in_off = t.open_off[P];
    in_cnt = t.open_cnt[P];
  }
  const bool cached = in_cnt <= 64;
  if (!WRITE) ncand = 0;
  if (WRITE && cached) {
    const int total = min(ncand, TRAV_CAND);
    for (int cb = 0; cb < total; cb += 64) {
      if (sp > TRAV_STACK - TRAV_RESERVE - 512) drain<WRITE>(t, S, L, sp, open_out, th2, eps, pairs);
      const bool valid = cb + lane < total;
      const int C = valid ? L.cand[cb + lane] : 0;
      const int code = valid ? L.ccat[cb + lane] : 0;
#pragma unroll
      for (int tg = 0; tg < 8; ++tg) {
        if (tg < S.n) {
          const int cat = (code >> (3 * tg)) & 7;
          emit<WRITE>(t, S, tg, cat, valid, C, 0, open_out, pairs);
          if (S.leaf[tg]) push_item(t, L, sp, cat == CAT_DEEPEN, tg, C);
        }
      }
    }
    drain<WRITE>(t, S, L, sp, open_out, th2, eps, pairs);
    return;
  }
  for (int eb = 0; eb < in_cnt; eb += 64) {
    // expand 64 open-list entries into candidate cells (children, or the leaf itself)
    const int e = eb + lane;
    int ec = 0, c0 = 0;
    if (e < in_cnt) {
      if (l == 0) {
        ec = 1;  // the pair (root, root) of this request's tree
        c0 = P;
      } else {
        const int B = open_in[in_off + e];
        const int nB = t.nnchild[B];
        ec = nB > 0 ? nB : 1;
        c0 = nB > 0 ? t.nchild0[B] : B;
      }
    }
    int total;
    const int pos = wave_excl_scan_int(ec, &total);
    for (int q = 0; q < ec; ++q) L.cand[pos + q] = c0 + q;
    if (!WRITE && cached) ncand = total;
    __builtin_amdgcn_wave_barrier();
    for (int cb = 0; cb < total; cb += 64) {
      // a chunk pushes at most 64 items per target, 512 in all, and must leave
      // the depth-first reserve free
      if (sp > TRAV_STACK - TRAV_RESERVE - 512) drain<WRITE>(t, S, L, sp, open_out, th2, eps, pairs);
      const bool valid = cb + lane < total;
      const int C = valid ? L.cand[cb + lane] : 0;
      double4 gC = make_double4(0, 0, 0, 0);
      int nC = 0, npC = 0;
      if (valid) {
        gC = t.ngeo[C];
        nC = t.nnchild[C];
        npC = t.nend[C] - t.nbeg[C];
      }
      int code = 0;
#pragma unroll
      for (int tg = 0; tg < 8; ++tg) {
        if (tg < S.n) {
          const int cat = valid ? classify(S.id[tg], L.geo[tg], S.leaf[tg], C, gC, nC == 0, th2,
                                           eps)
                                : CAT_NONE;
          code |= cat << (3 * tg);
          emit<WRITE>(t, S, tg, cat, valid, C, npC, open_out, pairs);
          if (S.leaf[tg]) push_item(t, L, sp, cat == CAT_DEEPEN, tg, C);
        }
      }
      if (!WRITE && cached && valid) L.ccat[cb + lane] = code;
    }
    __builtin_amdgcn_wave_barrier();
  }
  drain<WRITE>(t, S, L, sp, open_out, th2, eps, pairs);
}

// Level l >= 1: one wavefront per cell P of level l-1 with children; the
// children are the targets.  Level 0: one wavefront per request root, whose
// only candidate is itself, so cells of different requests never meet.
__device__ void walk_parent(const DevTree &t, int l, int P, double th2, double eps, WaveLds &L) {
  const int lane = threadIdx.x & 63;
  Header *h = t.hdr;
  Sibs S;
  if (l == 0) {
    // a request's root is the only target of its group; every sibling slot
    // must hold a valid id because the slots are read below before the S.n
    // guard applies
    S.n = 1;
#pragma unroll
    for (int tg = 0; tg < 8; ++tg) S.id[tg] = P;
  } else {
    const int nc = t.nnchild[P];
    if (nc == 0) return;
    S.n = nc;
    const int c0 = t.nchild0[P];
#pragma unroll
    for (int tg = 0; tg < 8; ++tg) S.id[tg] = c0 + (tg < nc ? tg : 0);
  }
#pragma unroll
  for (int tg = 0; tg < 8; ++tg) {
    const int A = S.id[tg];
    S.leaf[tg] = t.nnchild[A] == 0;
    S.np[tg] = t.nend[A] - t.nbeg[A];
  }
  if (lane < 8) {
    int A = S.id[0];
    bool lf = S.leaf[0];
#pragma unroll
    for (int tg = 1; tg < 8; ++tg)
      if (lane == tg) {
        A = S.id[tg];
        lf = S.leaf[tg];
      }
    L.geo[lane] = t.ngeo[A];
    L.sid[lane] = A;
    L.sleaf[lane] = lf ? 1 : 0;
  }
  __builtin_amdgcn_wave_barrier();
  const int *open_in = (l & 1) ? t.open_buf0 : t.open_buf1;
  int *open_out = (l & 1) ? t.open_buf1 : t.open_buf0;
  unsigned long long pairs = 0;
  int ncand = 0;
  walk_group<false>(t, l, P, S, L, open_in, open_out, th2, eps, pairs, ncand);
  // allocate every target's lists (lane tg handles target tg)
  int mine[3] = {0, 0, 0};
#pragma unroll
  for (int tg = 0; tg < 8; ++tg)
    if (lane == tg)
#pragma unroll
      for (int k = 0; k < 3; ++k) mine[k] = S.cnt[tg][k];
  // one allocation per wavefront and list (the targets' lists laid out in
  // target order inside it): all wavefronts of a level allocate at about the
  // same time, and device-scope atomics on one address serialise
  int o[3] = {0, 0, 0};
  int bits = 0;
  {
    unsigned *const cur[3] = {&h->m2l_cursor, &h->p2p_cursor, &h->open_cursor[l]};
    const int64_t cap[3] = {t.cap_m2l, t.cap_p2p, t.cap_open};
    const int ovf_bit[3] = {OVF_M2L, OVF_P2P, OVF_OPEN};
    int incl[3], tot[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      incl[k] = mine[k];  // inclusive prefix over the target lanes 0..7
#pragma unroll
      for (int d = 1; d < 8; d <<= 1) {
        const int y = __shfl_up(incl[k], d, 64);
        if (lane >= d) incl[k] += y;
      }
      tot[k] = __shfl(incl[k], 7, 64);
    }
    // lane k allocates list k: the three in one instruction, one round trip
    const int tk = lane == 0 ? tot[0] : lane == 1 ? tot[1] : tot[2];
    int got = 0;
    if (lane < 3 && tk > 0) got = (int)atomicAdd(lane == 0 ? cur[0] : lane == 1 ? cur[1] : cur[2],
                                                 (unsigned)tk);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int base = __shfl(got, k, 64);
      o[k] = base + incl[k] - mine[k];
      if (lane < S.n && (int64_t)base + tot[k] > cap[k]) bits |= ovf_bit[k];
    }
  }
  // if any target's lists do not fit, the wavefront writes none of them and
  // every one of its targets gets empty lists: no count ever covers entries
  // that were not written (the host regrows and rebuilds)
  const bool ovf = __ballot(bits != 0) != 0ull;
  if (lane < S.n) {
    int A = S.id[0];
#pragma unroll
    for (int tg = 1; tg < 8; ++tg)
      if (lane == tg) A = S.id[tg];
    t.m2l_off[A] = o[0];
    t.m2l_cnt[A] = ovf ? 0 : mine[0];
    t.p2p_off[A] = o[1];
    t.p2p_cnt[A] = ovf ? 0 : mine[1];
    t.open_off[A] = o[2];
    t.open_cnt[A] = ovf ? 0 : mine[2];
    if (bits) atomicOr(&h->overflow, bits);
  }
  if (ovf) return;
#pragma unroll
  for (int tg = 0; tg < 8; ++tg)
#pragma unroll
    for (int k = 0; k < 3; ++k) S.off[tg][k] = __shfl(o[k], tg, 64);
  walk_group<true>(t, l, P, S, L, open_in, open_out, th2, eps, pairs, ncand);
  pairs = wave_sum(pairs);
  if (lane == 0 && pairs) atomicAdd(&h->p2p_pairs, pairs);
}

__global__ __launch_bounds__(TRAV_WAVES * 64) void k_walk_level(DevTree t, int l, int ps, int pe,
                                                                double th2, double eps) {
  __shared__ WaveLds lds[TRAV_WAVES];
  const int w = threadIdx.x >> 6;
  const int P = ps + xcd_block<32>(blockIdx.x, gridDim.x) * TRAV_WAVES + w;
  if (P >= pe) return;
  walk_parent(t, l, P, th2, eps, lds[w]);
}

// Level l with its bounds read from the tree header (queued before the
// level sizes are known on the host): the waves of the grid stride over the
// parents; nothing is done on a tree whose node workspace overflowed.
__global__ __launch_bounds__(TRAV_WAVES * 64) void k_walk_level_dev(DevTree t, int l, double th2,
                                                                    double eps) {
  __shared__ WaveLds lds[TRAV_WAVES];
  const Header *h = t.hdr;
  if (h->overflow & OVF_NODES) return;
  const int ps = l == 0 ? 0 : h->lvl_start[l - 1];
  const int pe = l == 0 ? t.n_req : h->lvl_start[l];
  const int w = threadIdx.x >> 6;
  const int nw = gridDim.x * TRAV_WAVES;
  for (int P = ps + xcd_block<32>(blockIdx.x, gridDim.x) * TRAV_WAVES + w; P < pe; P += nw)
    walk_parent(t, l, P, th2, eps, lds[w]);
}

// All levels of the walk in one workgroup (small trees): the waves share the
// parents of a level, and a barrier separates levels (a level reads the open
// lists the previous one wrote).  Level sizes come from the tree header.
__global__ __launch_bounds__(SMALL_THREADS) void k_walk_small(DevTree t, double th2, double eps) {
  __shared__ WaveLds lds[SMALL_WAVES];
  const int w = threadIdx.x >> 6;
  const Header *h = t.hdr;
  for (int l = 0; l <= FMM_MAXLEVEL; ++l) {
    const int ps = l == 0 ? 0 : h->lvl_start[l - 1];
    const int pe = l == 0 ? t.n_req : h->lvl_start[l];
    if (l > 0 && h->lvl_start[l + 1] <= h->lvl_start[l]) break;  // no cells at level l
    for (int P = ps + w; P < pe; P += SMALL_WAVES) walk_parent(t, l, P, th2, eps, lds[w]);
    __syncthreads();
  }
}

__global__ void k_reset_lists(Header *h) {
  int i = threadIdx.x;
  if (i == 0) {
    h->m2l_cursor = 0;
    h->p2p_cursor = 0;
    h->p2p_pairs = 0;
    h->overflow &= OVF_NODES | OVF_DEPTH;
  }
  if (i < FMM_NLEVELS) h->open_cursor[i] = 0;
}

hipError_t launch_reset_lists(const DevTree &t, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_lists, dim3(1), dim3(64), 0, s, t.hdr);
  return hipGetLastError();
}

hipError_t launch_traverse_small(const DevTree &t, const BuildArgs &a, hipStream_t s) {
  launch_reset_lists(t, s);
  if (a.n <= 0) return hipGetLastError();
  if (a.tm) a.tm->start(PH_WALK, s);
  hipLaunchKernelGGL(k_walk_small, dim3(1), dim3(SMALL_THREADS), 0, s, t, a.theta * a.theta,
                     a.eps);
  if (a.tm) a.tm->stop(s);
  return hipGetLastError();
}

hipError_t launch_traverse(const DevTree &t, const BuildArgs &a, hipStream_t s) {
  launch_reset_lists(t, s);
  if (a.n <= 0) return hipGetLastError();
  const double th2 = a.theta * a.theta;
  if (a.tm) a.tm->start(PH_WALK, s);
  for (int l = 0; l <= a.depth; ++l) {
    int ps = l == 0 ? 0 : a.lvl_host[l - 1];
    int pe = l == 0 ? a.n_req : a.lvl_host[l];
    int nw = pe - ps;
    if (nw <= 0) continue;
    hipLaunchKernelGGL(k_walk_level, dim3((nw + TRAV_WAVES - 1) / TRAV_WAVES),
                       dim3(TRAV_WAVES * 64), 0, s, t, l, ps, pe, th2, a.eps);
  }
  if (a.tm) a.tm->stop(s);
  return hipGetLastError();
}

// Levels 0..levels with the bounds of each read on the device (see
// k_walk_level_dev); the grid fills the chip for large trees.
hipError_t launch_traverse_dev(const DevTree &t, const BuildArgs &a, int levels, hipStream_t s) {
  launch_reset_lists(t, s);
  if (a.n <= 0) return hipGetLastError();
  const double th2 = a.theta * a.theta;
  const int blocks = std::min(2048, std::max(16, a.n / 512));
  if (a.tm) a.tm->start(PH_WALK, s);
  for (int l = 0; l <= levels && l <= FMM_MAXLEVEL; ++l)
    hipLaunchKernelGGL(k_walk_level_dev, dim3(blocks), dim3(TRAV_WAVES * 64), 0, s, t, l, th2,
                       a.eps);
  if (a.tm) a.tm->stop(s);
  return hipGetLastError();
}
