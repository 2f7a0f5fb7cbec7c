// Internal declarations shared by the HIP translation units of libfmm355.
//
// Data layout in HBM (one context, capacities fixed at creation):
//   particles (Morton-sorted order, SoA):  keys u64, slot i32 (active slot of
//     the particle), positions f64 x3, cell-local offsets f32 x3, masses f64 and
//     f32, leaf id i32, near-field (P2P) results f64 x4;
//   nodes (level-major: all level-0 nodes, then level 1, ...; inside a level in
//     Morton order): begin/end/level/parent/first-child/child-count i32,
//     geometry double4 (centre xyz, half side), multipole and local
//     coefficient rows of K = C(p+3,3) reals (node-major);
//   interaction lists: per target node (offset, count) into flat i32 arrays of
//     source node ids (directed entries; the unordered pair {A,B} appears once
//     in A's list and once in B's list).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define FMM_MAXLEVEL 21
#define FMM_NLEVELS (FMM_MAXLEVEL + 1)
#define FMM_BLOCK 256
#define FMM_SCAN_BLOCKS 256
#define FMM_BBOX_BLOCKS 256  // box-reduction blocks per request, at most
#define SORT_TILE 4096       // keys per radix-sort tile (one histogram column)
#define SORT_RAW_TILES 16    // sorts of at most this many tiles run without digit-scan launches
#define SORT_MAX_PASSES 12   // 8 key digits + at most 4 request digits
// single-workgroup ("small") build, walk and level passes
#define SMALL_WAVES 8
#define SMALL_THREADS (SMALL_WAVES * 64)
#define SMALL_N (SMALL_THREADS * 16)  // active particles of a batch, at most
#define SMALL_AUTO_N 1024             // the small path's default reach (beyond it the
                                      // multi-workgroup path is faster)
#define SMALL_NODES 2048              // cells of a tree whose M2M / L2L levels run in one workgroup

// error bits latched in Header::overflow
#define OVF_NODES 1
#define OVF_M2L 2
#define OVF_P2P 4
#define OVF_OPEN 8
#define OVF_STACK 16
// the tree holds cells deeper than the levels the (predicted) walk covers: the
// cells below them have no lists, so nothing may be evaluated on it
#define OVF_DEPTH 32

struct Header {
  int32_t lvl_start[FMM_NLEVELS + 2];  // nodes of level l: [lvl_start[l], lvl_start[l+1])
  uint32_t m2l_cursor;                 // ordered M2L entries written (or needed)
  uint32_t p2p_cursor;                 // ordered P2P entries written (or needed)
  uint32_t open_cursor[FMM_NLEVELS];   // open-list entries per level
  int32_t overflow;                    // OVF_* bits
  int32_t nonfinite;                   // an input position was not finite
  unsigned long long p2p_pairs;        // ordered particle interactions in P2P
  int32_t n_leaves;
  int32_t max_prefix;  // deepest level of a cell holding more than leaf_size particles
};

// Box: o[3] (origin), L (side), s = 2^21/L, lo[3], hi[3]
struct Box {
  double o[3];
  double L;
  double s;
  double lo[3];
  double hi[3];
};

// One independent particle system of a batched solve.  Its active particles
// occupy slots [off, off + n) of the batch; positions/masses are read through
// its own pointers, outputs written to its own acc/pot.
struct DevReq {
  const double *pos;      // 3 x n_total SoA
  const int32_t *active;  // n indices or NULL
  const double *mass;     // n_total
  double *acc;            // 3 x n SoA
  double *pot;            // n
  const uint8_t *sinks;   // n flags, or NULL: every particle is a sink
  int64_t n_total;
  int32_t off;
  int32_t n;
};

struct DevTree {
  // batch of requests (R = 1 for a plain solve)
  DevReq *reqs;       // [cap_req]
  int32_t *req_off;   // [cap_req + 1] slot offsets
  int32_t *blk_off;   // [cap_req + 1] first bbox block of each request
  int32_t *slot_req;  // [cap_n] request of each slot
  int32_t *nreq;      // [cap_nodes] request of each cell
  int n_req;
  int cap_req;
  // particles, sorted order
  uint64_t *key, *key2;
  int32_t *slot, *slot2;
  double *sx, *sy, *sz;
  double *sm;
  float *sm32;
  int32_t *leaf_of;
  double *near;  // [4][cap_n]: ax, ay, az, pot
  double4 *pak;  // [cap_n] positions packed per active slot by the key pass, so
                 // that the sorted gather reads one 32-byte record per particle
  // nodes
  int32_t *nbeg, *nend, *nlev, *nparent, *nchild0, *nnchild;
  double4 *ngeo;
  int32_t *bounds;  // [cap_nodes][8]
  void *M, *L;      // [cap_nodes][Kmax] of float or double
  void *Mh;         // [cap_nodes][KHmax]: moments folded onto z-degree <= 1 (harmonic far field)
  // lists
  int32_t *m2l_off, *m2l_cnt, *m2l_src;
  int32_t *p2p_off, *p2p_cnt, *p2p_src;
  int32_t *open_off, *open_cnt;
  int32_t *open_buf0, *open_buf1;
  // scratch
  int32_t *scan_part;          // [FMM_SCAN_BLOCKS]
  double *bbox_part;           // [bbox blocks][6]
  uint32_t *sort_hist;         // [256][sort blocks]
  uint32_t *sort_dtot;         // [256] digit totals
  uint32_t *scan_blk;          // block sums of the generic scan
  Header *hdr;
  Box *box;  // [cap_req]
  int64_t cap_n, cap_nodes, cap_m2l, cap_p2p, cap_open;
  int kmax, khmax;
};

// ---------------------------------------------------------------------------
// wavefront helpers (wave64)
// ---------------------------------------------------------------------------
// largest r in [0, m) with off[r] <= x (request of a slot, or of a sorted
// position: both lie in the request's [off[r], off[r + 1]))
__device__ __forceinline__ int upper_index(const int32_t *off, int m, int x) {
  int lo = 0, hi = m - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= x)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ unsigned long long lanes_below_mask() {
  int l = __lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Workgroups are dealt to the 8 XCDs (each with its own L2) round-robin in
// blockIdx order.  xcd_block maps blockIdx to a logical block index so that
// each XCD runs chunks of C consecutive logical blocks (the chunks themselves
// dealt round-robin): neighbouring cells, which share most of their sources,
// meet in one L2, while every XCD still gets a mix of the whole range.  A
// bijection on [0, G): the blocks past the last whole round of 8 C keep their
// index.
#define FMM_XCDS 8
template <int C>
__device__ __forceinline__ int xcd_block(int b, int G) {
  const int full = G / (FMM_XCDS * C) * (FMM_XCDS * C);
  if (b >= full) return b;
  const int x = b % FMM_XCDS, k = b / FMM_XCDS;
  return ((k / C) * FMM_XCDS + x) * C + k % C;
}

__device__ __forceinline__ int wave_excl_scan_int(int v, int *total) {
  // inclusive Hillis-Steele over 64 lanes
  int x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int y = __shfl_up(x, off, 64);
    if (__lane_id() >= off) x += y;
  }
  *total = __shfl(x, 63, 64);
  return x - v;
}

// ---------------------------------------------------------------------------
// per-phase HIP-event timing on the context's stream (off unless enabled)
// ---------------------------------------------------------------------------
enum {
  PH_SORT = 0,   // root box, keys, radix sort, sorted gather
  PH_TREE = 1,   // level-by-level split, leaf marking
  PH_WALK = 2,   // symmetric dual walk
  PH_UP = 3,     // mass gather, P2M, M2M
  PH_M2L = 4,
  PH_P2P = 5,
  PH_DOWN = 6,   // L2L, L2P
  PH_N = 7
};

struct PhaseTimer {
  static const int CAP = 512;
  bool on = false;
  bool ready = false;
  unsigned mask = ~0u;  // phases recorded (bit p for phase p)
  hipEvent_t a[CAP], b[CAP];
  int ph[CAP];
  int n = 0, cur = -1;
  double ms[PH_N] = {0};
  long long cnt[PH_N] = {0};
  // an interval of phase p on stream s (intervals on different streams may overlap)
  int begin(int p, hipStream_t s) {
    if (!on || !(mask >> p & 1u)) return -1;
    if (n == CAP) flush();
    hipEventRecord(a[n], s);
    ph[n] = p;
    return n++;
  }
  void end(int k, hipStream_t s) {
    if (on && k >= 0) hipEventRecord(b[k], s);
  }
  void start(int p, hipStream_t s) { cur = begin(p, s); }
  void stop(hipStream_t s) {
    end(cur, s);
    cur = -1;
  }
  void flush() {
    for (int i = 0; i < n; ++i) {
      float t = 0.f;
      hipEventSynchronize(b[i]);
      hipEventElapsedTime(&t, a[i], b[i]);
      ms[ph[i]] += t;
      cnt[ph[i]] += 1;
    }
    n = 0;
  }
};

// ---------------------------------------------------------------------------
// host-side launchers (one translation unit each)
// ---------------------------------------------------------------------------
struct BuildArgs {
  int n;          // active particles over all requests
  int n_req;      // requests (roots)
  int n_blk;      // bbox blocks over all requests
  int leaf_size;
  double eps;
  double theta;
  PhaseTimer *tm;
  const int32_t *lvl_host;  // level starts of the built tree (host copy), for the walk
  int depth;
};

// tree.hip
hipError_t launch_sort(const DevTree &t, const BuildArgs &a, hipStream_t s);
// whole build up to the walk in one workgroup (a.n <= SMALL_N)
hipError_t launch_build_small(const DevTree &t, const BuildArgs &a, hipStream_t s);
hipError_t launch_build_tree(const DevTree &t, const BuildArgs &a, int max_level, hipStream_t s);
// every split level in a fixed number of launches (no host read of the split
// depth first); only for leaf sizes up to the window kept in LDS
bool build_tree_direct_ok(int leaf_size);
hipError_t launch_build_tree_direct(const DevTree &t, const BuildArgs &a, int walk_levels,
                                    hipStream_t s);
// traverse.hip
hipError_t launch_traverse(const DevTree &t, const BuildArgs &a, hipStream_t s);
// levels 0..levels, level bounds read on the device (tree sizes not yet known)
hipError_t launch_traverse_dev(const DevTree &t, const BuildArgs &a, int levels, hipStream_t s);
// all walk levels in one workgroup, level sizes read on the device
hipError_t launch_traverse_small(const DevTree &t, const BuildArgs &a, hipStream_t s);
hipError_t launch_reset_lists(const DevTree &t, hipStream_t s);
// eval.hip
struct EvalArgs {
  hipStream_t side;         // P2P runs here, concurrently with the multipole passes
  hipEvent_t fork, join;
  int n;
  int n_nodes;
  int p;
  int kernel;     // 0 Wendland, 1 Plummer
  int mixed;      // 0 FP64, 1 mixed
  double eps;
  const int32_t *lvl_start_host;  // host copy, FMM_NLEVELS+1 entries
  int depth;
  PhaseTimer *tm;
  // queued before the host read the tree header: n_nodes, lvl_start_host and
  // depth are estimates (grid sizes, loop bounds) and the kernels take the
  // tree's sizes from the header
  bool dev;
  // with dev: n_nodes, lvl_start_host and depth are the tree's exact sizes (the
  // tree is final, only the lists may have overflowed): grids are exact, and
  // the kernels still take the sizes from the header and skip an overflowed build
  bool exact;
  // mass gather, P2M and M2M already queued by launch_upward (on the side
  // stream, beside the walk); the main stream waits for up_done before M2L
  bool upward_done;
  hipEvent_t up_done;
};
hipError_t launch_evaluate(const DevTree &t, const EvalArgs &e, hipStream_t s);
// mass gather, P2M and M2M of an evaluation on stream s (exact tree sizes)
hipError_t launch_upward(const DevTree &t, const EvalArgs &e, hipStream_t s);
bool eval_order_supported(int p);
// grad.hip: force gradient of one system's n active particles (SoA 6 x n) on
// the tree and local expansions of the evaluation just queued on stream s
hipError_t launch_force_gradient(const DevTree &t, int n_nodes, int n, int p, int kernel,
                                 bool mixed, double eps, double *stage, double *grad,
                                 hipStream_t s);
// vector-source pass (eval.hip): sources m_j v_j on the last build's tree (one
// system), vec SoA 3 x e.n in active order, dv scratch 3 x cap_n doubles;
// the request's acc receives +gradient of their potential, pot the potential
hipError_t launch_dipole(const DevTree &t, const EvalArgs &e, const double *vec, double *dv,
                         hipStream_t s);
// its near field (grad.hip): minus sum_j m_j H(x_i - x_j) v_j over the P2P
// partners into near[0..2], sum_j m_j v_j . grad psi(x_i - x_j) into near[3]
hipError_t launch_p2p_dipole(const DevTree &t, int n_nodes, int kernel, bool mixed, double eps,
                             const double *dv, hipStream_t s);
// hhs.hip
hipError_t launch_gather_mask_mass(const double *mass, const int32_t *sys, int n_sys,
                                   const int32_t *flag_fast, int mask_fast, double *out,
                                   hipStream_t s);
