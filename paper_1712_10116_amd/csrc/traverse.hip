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
// a per-wavefront LDS stack.  One wavefront handles one target cell; level l
// of the tree is one launch.  Outputs are written in two passes (count, then
// write after an atomic allocation), so each cell's lists are contiguous and
// their content and order are deterministic.
//
// Well-separation is Eq. (1) with R = half side, plus the softening rule of
// Sec. 2.3, written in IEEE double without contraction:
//   d2 = (dx*dx + dy*dy) + dz*dz,  S = hA + hB,
//   d2*(theta*theta) > S*S  and  d2 > (eps + sqrt(3)*S)^2.
#include "common.h"

#define TRAV_WAVES 4
#define TRAV_STACK 2048

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

struct TravOut {
  int *m2l, *p2p, *open;
  int om2l, op2p, oopen;
  int wm, wp, wo;
  unsigned long long pairs;
};

// Classify candidate C of target A and (pass 1) emit it; returns the number
// of children to push for a descending leaf target.
template <bool WRITE>
__device__ __forceinline__ void classify_emit(const DevTree &t, int A, double4 gA, bool leafA,
                                              int nA, bool valid, int C, double th2, double eps,
                                              int &cm2l, int &cp2p, int &copen, TravOut &o,
                                              int *stk, int &sp) {
  int cat = CAT_NONE;
  int nC = 0;
  if (valid) {
    nC = t.nnchild[C];
    if (C == A)
      cat = leafA ? CAT_P2P : CAT_OPEN;
    else if (well_separated(gA, t.ngeo[C], th2, eps))
      cat = CAT_M2L;
    else if (leafA)
      cat = nC == 0 ? CAT_P2P : CAT_DEEPEN;
    else
      cat = CAT_OPEN;
  }
  const unsigned long long below = lanes_below_mask();
  unsigned long long bm = __ballot(cat == CAT_M2L);
  unsigned long long bp = __ballot(cat == CAT_P2P);
  unsigned long long bo = __ballot(cat == CAT_OPEN);
  if (WRITE) {
    if (cat == CAT_M2L) o.m2l[o.om2l + o.wm + __popcll(bm & below)] = C;
    if (cat == CAT_P2P) {
      o.p2p[o.op2p + o.wp + __popcll(bp & below)] = C;
      int nCp = t.nend[C] - t.nbeg[C];
      o.pairs += (unsigned long long)nA * (unsigned long long)nCp - (C == A ? (unsigned)nA : 0u);
    }
    if (cat == CAT_OPEN) o.open[o.oopen + o.wo + __popcll(bo & below)] = C;
    o.wm += __popcll(bm);
    o.wp += __popcll(bp);
    o.wo += __popcll(bo);
  }
  cm2l += __popcll(bm);
  cp2p += __popcll(bp);
  copen += __popcll(bo);
  // push the children of descending candidates
  int push = cat == CAT_DEEPEN ? nC : 0;
  int total;
  int pos = wave_excl_scan_int(push, &total);
  if (total) {
    if (sp + total > TRAV_STACK) {
      // drop the descent (the build reports the overflow as an error); sp only
      // ever covers entries that were written
      if (__lane_id() == 0) atomicOr(&t.hdr->overflow, OVF_STACK);
    } else {
      if (push) {
        int c0 = t.nchild0[C];
        for (int k = 0; k < push; ++k) stk[sp + pos + k] = c0 + k;
      }
      sp += total;
    }
  }
}

template <bool WRITE>
__device__ void walk_target(const DevTree &t, int l, int A, const int *open_in, TravOut &o,
                            int *stk, double th2, double eps, int &cm2l, int &cp2p, int &copen) {
  const int lane = __lane_id();
  const double4 gA = t.ngeo[A];
  const bool leafA = t.nnchild[A] == 0;
  const int nA = t.nend[A] - t.nbeg[A];
  int in_off = 0, in_cnt = 1;
  if (l > 0) {
    int P = t.nparent[A];
    in_off = t.open_off[P];
    in_cnt = t.open_cnt[P];
  }
  int sp = 0;
  cm2l = cp2p = copen = 0;
  for (int base = 0; base < in_cnt; base += 64) {
    int ei = base + lane;
    bool valid = ei < in_cnt;
    int ec = 0, c0 = 0;
    if (valid) {
      if (l == 0) {
        ec = 1;
        c0 = 0;  // the pair (root, root)
      } else {
        int B = open_in[in_off + ei];
        int nB = t.nnchild[B];
        ec = nB > 0 ? nB : 1;
        c0 = nB > 0 ? t.nchild0[B] : B;
      }
    }
    for (int k = 0; k < 8; ++k) {
      bool has = k < ec;
      if (__ballot(has) == 0ull) break;
      classify_emit<WRITE>(t, A, gA, leafA, nA, has, c0 + k, th2, eps, cm2l, cp2p, copen, o, stk,
                           sp);
    }
  }
  // descend candidates of a leaf target (LIFO, up to 64 at a time)
  while (sp > 0) {
    int take = min(sp, 64);
    bool valid = lane < take;
    int C = valid ? stk[sp - take + lane] : 0;
    __builtin_amdgcn_wave_barrier();
    sp -= take;
    classify_emit<WRITE>(t, A, gA, leafA, nA, valid, C, th2, eps, cm2l, cp2p, copen, o, stk, sp);
    __builtin_amdgcn_wave_barrier();
  }
}

__global__ __launch_bounds__(TRAV_WAVES * 64) void k_traverse_level(DevTree t, int l, double th2,
                                                                     double eps) {
  __shared__ int stack[TRAV_WAVES][TRAV_STACK];
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  Header *h = t.hdr;
  if (h->overflow & OVF_NODES) return;  // child ids may lie beyond the node arrays
  const int s = h->lvl_start[l], e = min(h->lvl_start[l + 1], (int)t.cap_nodes);
  const int *open_in = (l & 1) ? t.open_buf0 : t.open_buf1;
  int *open_out = (l & 1) ? t.open_buf1 : t.open_buf0;
  unsigned long long pairs = 0;
  for (int A = s + blockIdx.x * TRAV_WAVES + w; A < e; A += gridDim.x * TRAV_WAVES) {
    TravOut o;
    o.m2l = t.m2l_src;
    o.p2p = t.p2p_src;
    o.open = open_out;
    o.wm = o.wp = o.wo = 0;
    o.pairs = 0;
    int cm, cp, co;
    walk_target<false>(t, l, A, open_in, o, stack[w], th2, eps, cm, cp, co);
    int om = 0, op = 0, oo = 0;
    if (lane == 0) {
      om = (int)atomicAdd(&h->m2l_cursor, (unsigned)cm);
      op = (int)atomicAdd(&h->p2p_cursor, (unsigned)cp);
      oo = (int)atomicAdd(&h->open_cursor[l], (unsigned)co);
    }
    om = __shfl(om, 0, 64);
    op = __shfl(op, 0, 64);
    oo = __shfl(oo, 0, 64);
    bool ovf = (int64_t)om + cm > t.cap_m2l || (int64_t)op + cp > t.cap_p2p ||
               (int64_t)oo + co > t.cap_open;
    if (lane == 0) {
      t.m2l_off[A] = om;
      t.m2l_cnt[A] = ovf ? 0 : cm;
      t.p2p_off[A] = op;
      t.p2p_cnt[A] = ovf ? 0 : cp;
      t.open_off[A] = oo;
      t.open_cnt[A] = ovf ? 0 : co;
      if (ovf) {
        int bits = 0;
        if ((int64_t)om + cm > t.cap_m2l) bits |= OVF_M2L;
        if ((int64_t)op + cp > t.cap_p2p) bits |= OVF_P2P;
        if ((int64_t)oo + co > t.cap_open) bits |= OVF_OPEN;
        atomicOr(&h->overflow, bits);
      }
    }
    if (!ovf) {
      o.om2l = om;
      o.op2p = op;
      o.oopen = oo;
      walk_target<true>(t, l, A, open_in, o, stack[w], th2, eps, cm, cp, co);
      pairs += o.pairs;
    }
  }
  pairs = wave_sum(pairs);
  if (lane == 0 && pairs) atomicAdd(&h->p2p_pairs, pairs);
}

__global__ void k_reset_lists(Header *h) {
  int i = threadIdx.x;
  if (i == 0) {
    h->m2l_cursor = 0;
    h->p2p_cursor = 0;
    h->p2p_pairs = 0;
    h->overflow &= OVF_NODES;
  }
  if (i < FMM_NLEVELS) h->open_cursor[i] = 0;
}

hipError_t launch_reset_lists(const DevTree &t, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_lists, dim3(1), dim3(64), 0, s, t.hdr);
  return hipGetLastError();
}

hipError_t launch_traverse(const DevTree &t, const BuildArgs &a, hipStream_t s) {
  launch_reset_lists(t, s);
  if (a.n <= 0) return hipGetLastError();
  const double th2 = a.theta * a.theta;
  if (a.tm) a.tm->start(PH_WALK, s);
  for (int l = 0; l <= FMM_MAXLEVEL; ++l)
    hipLaunchKernelGGL(k_traverse_level, dim3(2048), dim3(TRAV_WAVES * 64), 0, s, t, l, th2,
                       a.eps);
  if (a.tm) a.tm->stop(s);
  return hipGetLastError();
}
