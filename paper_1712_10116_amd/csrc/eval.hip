// Mass-dependent passes of the FMM on gfx950: P2M, M2M (upward), M2L over
// each cell's symmetric interaction list, L2L (downward), P2P over each
// leaf's symmetric near list, L2P.  Templated on the working precision T of
// the expansions (double, or float for the mixed form) and the order P.
//
// Both sides of an unordered cell pair (A, B) evaluate it from their own
// list: D^k psi is odd/even under R -> -R exactly in IEEE arithmetic, and the
// particle pair kernel uses x_j - x_i = -(x_i - x_j) exactly, so the force of
// every pair on A is the negative of its force on B (Eq. (2) of the paper)
// while no two wavefronts ever write the same cell or particle.
//
// Mixed form: cell-local FP32 offsets (x - z_leaf) and the FP64 difference of
// the two leaf centres rounded once to FP32 give every particle separation;
// FP32 partial sums over blocks of 16 sources are added into FP64
// accumulators; expansions are FP32 on size-scaled coefficients.
#include "common.h"
#include "expansion.h"

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(FMM_BLOCK) void k_gather_mass(DevTree t, int n) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int s = t.slot[j];
  const DevReq q = t.reqs[upper_index(t.req_off, t.n_req, j)];
  if (!q.mass) return;  // system skipped in this evaluation
  const int i = s - q.off;
  int64_t g = q.active ? q.active[i] : i;
  double m = q.mass[g];
  t.sm[j] = m;
  t.sm32[j] = (float)m;
}

template <typename T, int P>
__device__ __forceinline__ void load_row(const T *__restrict__ base, int kmax, int node,
                                         T (&v)[MI<P>::K]) {
  const T *row = base + (size_t)node * kmax;
#pragma unroll
  for (int t = 0; t < MI<P>::K; ++t) v[t] = row[t];
}

template <typename T, int P>
__device__ __forceinline__ void store_row(T *__restrict__ base, int kmax, int node,
                                          const T (&v)[MI<P>::K]) {
  T *row = base + (size_t)node * kmax;
#pragma unroll
  for (int t = 0; t < MI<P>::K; ++t) row[t] = v[t];
}

// folded moments of a cell (harmonic far field), stride khmax
template <typename T, int P>
__device__ __forceinline__ void store_folded(const DevTree &t, int node, const T (&M)[MI<P>::K]) {
  T h[HI<P>::KH];
  fold_moments<T, P>(M, h);
  T *row = (T *)t.Mh + (size_t)node * t.khmax;
#pragma unroll
  for (int j = 0; j < HI<P>::KH; ++j) row[j] = h[j];
}

// a system whose mass pointer is NULL is skipped by this evaluation
__device__ __forceinline__ bool skipped(const DevTree &t, int node) {
  return t.reqs[t.nreq[node]].mass == nullptr;
}

// Whether leaf A (sorted particles bA .. bA+nA-1) holds a sink of its
// system's evaluation; every one does when the system has no sink flags.
// Called by a whole wavefront with A the same in every lane.
__device__ __forceinline__ bool has_sink(const DevTree &t, int A, int bA, int nA) {
  const DevReq &q = t.reqs[t.nreq[A]];
  if (!q.sinks) return true;
  bool any = false;
  for (int j = bA + (int)(threadIdx.x & 63); j < bA + nA; j += 64)
    any = any || q.sinks[t.slot[j] - q.off] != 0;
  return __ballot(any) != 0ull;
}

// Node range of an evaluation.  n >= 0: the host's count.  n < 0: queued
// before the host read the tree header (the tree is checked afterwards and
// the evaluation redone if it fails): the count comes from the header, and
// nothing is evaluated on a tree or lists whose build overflowed a
// workspace (node arrays, list buffers or descent stack).
__device__ __forceinline__ bool tree_incomplete(const DevTree &t) {
  return (t.hdr->overflow & (OVF_NODES | OVF_M2L | OVF_P2P | OVF_OPEN | OVF_STACK | OVF_DEPTH)) !=
         0;
}
__device__ __forceinline__ int node_count(const DevTree &t, int n) {
  if (n >= 0) return n;
  return tree_incomplete(t) ? 0 : min(t.hdr->lvl_start[FMM_NLEVELS], (int)t.cap_nodes);
}
// cells of one level: [s, e) from the host, or s = -1 - l for level l read
// from the header as above
__device__ __forceinline__ void level_range(const DevTree &t, int &s, int &e) {
  if (s >= 0) return;
  const int l = -1 - s;
  if (tree_incomplete(t)) {
    s = e = 0;
    return;
  }
  s = t.hdr->lvl_start[l];
  e = t.hdr->lvl_start[l + 1];
}

// Value of v in another lane of the same DPP row (CTRL: a DPP16 control).
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over each aligned group of 8 lanes, every lane of the group ending with
// the same value: quad swaps (lane ^ 1, lane ^ 2), then the mirror within 8
// lanes, which pairs a lane with one of the other quad.  The 8 lanes of the
// group must be active.
template <typename T>
__device__ __forceinline__ T sum8(T v) {
  v += dpp_f<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f<0x141>(v);  // row_half_mirror
  return v;
}

// Value of v from the lane a row-broadcast DPP control names (0x142: lane 15
// of each row into the next row; 0x143: lane 31 into rows 2 and 3), in the
// rows of ROWS; 0 in the other rows.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_bcast(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, false));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_bcast(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the whole wavefront, valid in lane 63: each row of 16 lanes is
// summed with DPP (quad swaps, mirror within 8, mirror within 16), then row 1
// adds row 0 and row 3 adds row 2 (lane 15 / 47 broadcast), and row 3 adds
// rows 0 + 1 (lane 31 broadcast).  No LDS traffic.  All 64 lanes must be
// active.
template <typename T>
__device__ __forceinline__ T wave_total_last(T v) {
  v += dpp_f<0xB1>(v);
  v += dpp_f<0x4E>(v);
  v += dpp_f<0x141>(v);
  v += dpp_f<0x140>(v);
  v += dpp_bcast<0x142, 0xA>(v);
  v += dpp_bcast<0x143, 0xC>(v);
  return v;
}

// The far-field cell kernels give each cell an aligned group of 8 lanes;
// g8 = lane & 7 is the lane's place in it.  Branches on the cell are uniform
// over the group, so its 8 lanes are active at every group sum.

// P2M at leaves: Mt[k] = sum_j m_j (u_j/h)^k/k!, lane g8 summing particles
// g8, g8 + 8, ... of the leaf (compensated in FP32, then the lanes' partial
// sums and compensations added in FP64 and rounded once).
template <typename T, int P>
__device__ __forceinline__ void p2m_cell8(const DevTree &t, int i, int g8, bool harm) {
  constexpr int K = MI<P>::K;
  T *M = (T *)t.M;
  if (t.nnchild[i] != 0 || skipped(t, i)) return;
  const double4 g = t.ngeo[i];
  const double ih = 1.0 / g.w;
  T acc[K], cmp[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = cmp[k] = T(0);
  for (int j = t.nbeg[i] + g8; j < t.nend[i]; j += 8) {
    t.leaf_of[j] = i;
    T mono[K];
    monomials<T, P>((T)((t.sx[j] - g.x) * ih), (T)((t.sy[j] - g.y) * ih),
                    (T)((t.sz[j] - g.z) * ih), mono);
    const T m = (T)t.sm[j];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (sizeof(T) == 4) {  // Kahan-Babuska summation of the FP32 moments
        T y = m * mono[k] - cmp[k];
        T s = acc[k] + y;
        cmp[k] = (s - acc[k]) - y;
        acc[k] = s;
      } else {
        acc[k] = fma(m, mono[k], acc[k]);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = (T)sum8<double>((double)acc[k] - (double)cmp[k]);
  if (g8 == 0) {
    store_row<T, P>(M, t.kmax, i, acc);
    if (harm) store_folded<T, P>(t, i, acc);
  }
}

template <typename T, int P>
__global__ __launch_bounds__(FMM_BLOCK) void k_p2m(DevTree t, int n_nodes, bool harm) {
  n_nodes = node_count(t, n_nodes);
  const int stride = (gridDim.x * blockDim.x) >> 3;
  for (int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 3; i < n_nodes; i += stride)
    p2m_cell8<T, P>(t, i, threadIdx.x & 7, harm);
}

// Moments of vector sources m_j v_j (the vector-source pass): the derivative
// of a leaf's mass moments along a displacement of each particle by its v_j,
// Mt[k] = -(m_j/h) sum_a v_a (u_j/h)^(k - e_a)/(k - e_a)!  (a with k_a >= 1),
// in the scaling of p2m_cell8.  dv: sorted-order SoA vectors, stride cap_n.
template <typename T, int P>
__device__ __forceinline__ void p2m_dip_cell8(const DevTree &t, const double *__restrict__ dv,
                                              int i, int g8, bool harm) {
  constexpr int K = MI<P>::K;
  constexpr MI<P> mi{};
  T *M = (T *)t.M;
  if (t.nnchild[i] != 0 || skipped(t, i)) return;
  const double4 g = t.ngeo[i];
  const double ih = 1.0 / g.w;
  const int64_t cap = t.cap_n;
  T acc[K], cmp[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = cmp[k] = T(0);
  for (int j = t.nbeg[i] + g8; j < t.nend[i]; j += 8) {
    t.leaf_of[j] = i;
    T mono[K];
    monomials<T, P>((T)((t.sx[j] - g.x) * ih), (T)((t.sy[j] - g.y) * ih),
                    (T)((t.sz[j] - g.z) * ih), mono);
    const double mh = t.sm[j] * ih;
    const T w[3] = {(T)(-mh * dv[j]), (T)(-mh * dv[cap + j]), (T)(-mh * dv[2 * cap + j])};
#pragma unroll
    for (int k = 0; k < K; ++k) {
      T v = T(0);
      if (mi.x[k] > 0) v = fma(w[0], mono[mi.at(mi.x[k] - 1, mi.y[k], mi.z[k])], v);
      if (mi.y[k] > 0) v = fma(w[1], mono[mi.at(mi.x[k], mi.y[k] - 1, mi.z[k])], v);
      if (mi.z[k] > 0) v = fma(w[2], mono[mi.at(mi.x[k], mi.y[k], mi.z[k] - 1)], v);
      if (sizeof(T) == 4) {  // Kahan-Babuska summation of the FP32 moments
        T y = v - cmp[k];
        T s = acc[k] + y;
        cmp[k] = (s - acc[k]) - y;
        acc[k] = s;
      } else {
        acc[k] += v;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = (T)sum8<double>((double)acc[k] - (double)cmp[k]);
  if (g8 == 0) {
    store_row<T, P>(M, t.kmax, i, acc);
    if (harm) store_folded<T, P>(t, i, acc);
  }
}

template <typename T, int P>
__global__ __launch_bounds__(FMM_BLOCK) void k_p2m_dip(DevTree t, int n_nodes,
                                                       const double *__restrict__ dv, bool harm) {
  const int stride = (gridDim.x * blockDim.x) >> 3;
  for (int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 3; i < n_nodes; i += stride)
    p2m_dip_cell8<T, P>(t, dv, i, threadIdx.x & 7, harm);
}

// Masses (as k_gather_mass) and the source vectors of the vector-source pass
// in sorted order: dv[a * cap + j] = vec[a * n + active slot of j] (one
// system, slots from 0).
__global__ __launch_bounds__(FMM_BLOCK) void k_gather_dip(DevTree t, int n,
                                                          const double *__restrict__ vec,
                                                          double *__restrict__ dv) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int s = t.slot[j];
  const DevReq q = t.reqs[0];
  const int64_t g = q.active ? q.active[s] : s;
  const double m = q.mass[g];
  t.sm[j] = m;
  t.sm32[j] = (float)m;
  const int64_t cap = t.cap_n;
  dv[j] = vec[s];
  dv[cap + j] = vec[n + s];
  dv[2 * cap + j] = vec[2 * n + s];
}

// M2M for a cell with children, lane g8 shifting child g8 (if any); the
// shifted children are summed over the group.
template <typename T, int P>
__device__ __forceinline__ void m2m_cell8(const DevTree &t, int i, int g8, bool harm) {
  constexpr int K = MI<P>::K;
  T *M = (T *)t.M;
  const int nc = t.nnchild[i];
  if (nc == 0 || skipped(t, i)) return;
  T acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = T(0);
  if (g8 < nc) {
    const double4 gp = t.ngeo[i];
    const double ih = 1.0 / gp.w;
    const int c = t.nchild0[i] + g8;
    const double4 gc = t.ngeo[c];
    T q[K], Mc[K];
    monomials<T, P>((T)((gc.x - gp.x) * ih), (T)((gc.y - gp.y) * ih), (T)((gc.z - gp.z) * ih),
                    q);
    load_row<T, P>(M, t.kmax, c, Mc);
    m2m_shift<T, P>(Mc, (T)(gc.w * ih), q, acc);
  }
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = sum8<T>(acc[k]);
  if (g8 == 0) {
    store_row<T, P>(M, t.kmax, i, acc);
    if (harm) store_folded<T, P>(t, i, acc);
  }
}

template <typename T, int P>
__global__ __launch_bounds__(FMM_BLOCK) void k_m2m(DevTree t, int s, int e, bool harm) {
  level_range(t, s, e);
  const int stride = (gridDim.x * blockDim.x) >> 3;
  for (int i = s + ((blockIdx.x * blockDim.x + threadIdx.x) >> 3); i < e; i += stride)
    m2m_cell8<T, P>(t, i, threadIdx.x & 7, harm);
}

// M2L: one wavefront per target cell A, lanes over A's list of sources B.
// With rho = h_A:  Lt_A[n] = (1/h_A) sum_m (-1)^|m| beta^|m| Mt_B[m]
//                             D^{n+m} psi_{eps/h_A}((zA - zB)/h_A),  beta = h_B/h_A.
// For the Wendland kernel the far field is exactly -1/r (the lists only hold
// pairs separated by more than eps), so the harmonic form is used: folded
// moments, contraction onto n_z <= 1, unfolding after the wave reduction.
template <typename T, int P, int KERNEL>
__global__ __launch_bounds__(FMM_BLOCK) void k_m2l(DevTree t, int n_nodes, double eps) {
  constexpr int K = MI<P>::K;
  constexpr int KH = HI<P>::KH;
  constexpr MI<P> mi{};
  constexpr HI<P> hi{};
  constexpr bool HARM = KERNEL == 0;
  const T *M = (const T *)t.M;
  const T *Mh = (const T *)t.Mh;
  T *L = (T *)t.L;
  const int lane = threadIdx.x & 63;
  const int wave = (xcd_block<32>(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) >> 6;
  const int nwaves = (gridDim.x * blockDim.x) >> 6;
  n_nodes = node_count(t, n_nodes);
  for (int A = wave; A < n_nodes; A += nwaves) {
    if (skipped(t, A)) continue;
    const double4 gA = t.ngeo[A];
    const double ih = 1.0 / gA.w;
    const T e2 = KERNEL == 1 ? (T)((eps * ih) * (eps * ih)) : T(0);
    const int off = t.m2l_off[A], cnt = t.m2l_cnt[A];
    T acc[K];  // in the harmonic form the n_z >= 2 entries are set by the unfolding
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (!HARM || mi.z[k] <= 1) acc[k] = T(0);
    // the next source's index is read one iteration ahead, so that the
    // loads of a source's geometry and moments do not wait on it
    int Bn = lane < cnt ? t.m2l_src[off + lane] : 0;
    for (int q = lane; q < cnt; q += 64) {
      const int B = Bn;
      if (q + 64 < cnt) Bn = t.m2l_src[off + q + 64];
      const double4 gB = t.ngeo[B];
      const T X = (T)((gA.x - gB.x) * ih), Y = (T)((gA.y - gB.y) * ih),
              Z = (T)((gA.z - gB.z) * ih);
      const T beta = (T)(gB.w * ih);
      T D[K];
      if (HARM) {
        derivatives<T, P, 2>(X, Y, Z, e2, D);
        T Ms[KH];
        const T *row = Mh + (size_t)B * t.khmax;
#pragma unroll
        for (int j = 0; j < KH; ++j) Ms[j] = row[j];
        T bp = T(1);
#pragma unroll
        for (int d = 0; d <= P; ++d) {
#pragma unroll
          for (int j = 0; j < KH; ++j)
            if (mi.deg[hi.full[j]] == d) Ms[j] *= (d & 1) ? -bp : bp;
          bp *= beta;
        }
        m2l_contract_h<T, P>(Ms, D, acc);
      } else {
        derivatives<T, P>(X, Y, Z, e2, D);
        T Ms[K];
        load_row<T, P>(M, t.kmax, B, Ms);
        T bp = T(1);
#pragma unroll
        for (int d = 0; d <= P; ++d) {
#pragma unroll
          for (int m = 0; m < K; ++m)
            if (mi.deg[m] == d) Ms[m] *= (d & 1) ? -bp : bp;
          bp *= beta;
        }
        m2l_contract<T, P>(Ms, D, acc);
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (!HARM || mi.z[k] <= 1) acc[k] = wave_total_last(acc[k]) * (T)ih;
    if (HARM) unfold_locals<T, P>(acc);
    if (lane == 63) store_row<T, P>(L, t.kmax, A, acc);
  }
}

// L2L for the cells of one level: Lt_c += shift of the parent's Lt
template <typename T, int P>
__device__ __forceinline__ void l2l_cell(const DevTree &t, int c) {
  constexpr int K = MI<P>::K;
  T *L = (T *)t.L;
  if (skipped(t, c)) return;
  const int p = t.nparent[c];
  const double4 gp = t.ngeo[p], gc = t.ngeo[c];
  const double ih = 1.0 / gp.w;
  T q[K], Lp[K], Lc[K];
  monomials<T, P>((T)((gc.x - gp.x) * ih), (T)((gc.y - gp.y) * ih), (T)((gc.z - gp.z) * ih), q);
  load_row<T, P>(L, t.kmax, p, Lp);
  load_row<T, P>(L, t.kmax, c, Lc);
  l2l_shift<T, P>(Lp, (T)(gc.w * ih), q, Lc);
  store_row<T, P>(L, t.kmax, c, Lc);
}

template <typename T, int P>
__global__ __launch_bounds__(FMM_BLOCK) void k_l2l(DevTree t, int s, int e) {
  level_range(t, s, e);
  for (int c = s + blockIdx.x * blockDim.x + threadIdx.x; c < e; c += gridDim.x * blockDim.x)
    l2l_cell<T, P>(t, c);
}

// Small trees: all M2M levels (deepest first) or all L2L levels (root first)
// in one workgroup, a barrier between levels.
template <typename T, int P>
__global__ __launch_bounds__(FMM_BLOCK) void k_m2m_small(DevTree t, int depth, bool harm,
                                                         bool dev) {
  const Header *h = t.hdr;
  if (dev && tree_incomplete(t)) return;
  for (int l = depth - 1; l >= 0; --l) {
    for (int i = h->lvl_start[l] + (threadIdx.x >> 3); i < h->lvl_start[l + 1];
         i += blockDim.x >> 3)
      m2m_cell8<T, P>(t, i, threadIdx.x & 7, harm);
    __syncthreads();
  }
}

template <typename T, int P>
__global__ __launch_bounds__(FMM_BLOCK) void k_l2l_small(DevTree t, int depth, bool dev) {
  const Header *h = t.hdr;
  if (dev && tree_incomplete(t)) return;
  for (int l = 1; l <= depth; ++l) {
    for (int c = h->lvl_start[l] + threadIdx.x; c < h->lvl_start[l + 1]; c += blockDim.x)
      l2l_cell<T, P>(t, c);
    __syncthreads();
  }
}

// L2P + near field + un-permute: one thread per Morton-sorted particle.
// sgn = 1 writes the acceleration, minus the gradient of the potential;
// sgn = -1 writes the gradient itself (the vector-source pass).
template <typename T, int P>
__global__ __launch_bounds__(FMM_BLOCK) void k_l2p(DevTree t, int n, bool dev, double sgn) {
  constexpr int K = MI<P>::K;
  const T *L = (const T *)t.L;
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  if (dev && tree_incomplete(t)) return;  // leaf_of not written for this tree
  // the system first: leaf_of is written only for systems this evaluation covers
  const DevReq q = t.reqs[upper_index(t.req_off, t.n_req, j)];
  if (!q.mass) return;
  const int s = t.slot[j];
  const int64_t i = s - q.off, nq = q.n;
  if (q.sinks && !q.sinks[i]) return;  // not a sink of this evaluation
  const int leaf = t.leaf_of[j];
  const double4 g = t.ngeo[leaf];
  const double ih = 1.0 / g.w;
  T mono[K], Lt[K];
  monomials<T, P>((T)((t.sx[j] - g.x) * ih), (T)((t.sy[j] - g.y) * ih), (T)((t.sz[j] - g.z) * ih),
                  mono);
  load_row<T, P>(L, t.kmax, leaf, Lt);
  T phi, gx, gy, gz;
  l2p_eval<T, P>(Lt, mono, phi, gx, gy, gz);
  const int64_t cap = t.cap_n;
  q.acc[i] = sgn * (t.near[j] - (double)gx * ih);
  q.acc[nq + i] = sgn * (t.near[cap + j] - (double)gy * ih);
  q.acc[2 * nq + i] = sgn * (t.near[2 * cap + j] - (double)gz * ih);
  q.pot[i] = t.near[3 * cap + j] + (double)phi;
}

// ---------------------------------------------------------------------------
// P2P: one wavefront per target leaf, lanes = (sink, phase) pairs in a layout
// chosen per leaf (below).
// ---------------------------------------------------------------------------
template <typename R, int KERNEL>
struct PairKernel {
  // For a source of mass m at squared distance r2: mg = m psi'(r)/r (the
  // acceleration factor) and t = -m psi(r) (the potential, sign flipped).
  // Plummer: psi = -(r2 + eps2)^(-1/2).  Wendland C2 (Eq. 8): psi = -1/r for
  // r >= eps, the polynomial in u = r/eps inside.
  __device__ __forceinline__ static void eval(R r2, R m, R eps2, R inv_eps, R inv_eps3, R &mg,
                                              R &t) {
    if (KERNEL == 1) {
      const R rinv = fast_rsqrt<R>(r2 + eps2);
      t = m * rinv;
      mg = t * (rinv * rinv);
    } else {
      const R rinv = fast_rsqrt<R>(r2);
      t = m * rinv;
      mg = t * (rinv * rinv);
      if (r2 < eps2) {
        R r = r2 > R(0) ? r2 * rinv : R(0);
        R u = r * inv_eps;
        R u2 = u * u;
        mg = m * (fma(fma(fma(fma(R(21), u, R(-90)), u, R(140)), u, R(-84)), u2, R(14)) * inv_eps3);
        t = m * (fma(u2, fma(fma(fma(fma(R(-3), u, R(15)), u, R(-28)), u, R(21)), u2, R(-7)),
                     R(3)) * inv_eps);
      }
    }
  }
};

// One wavefront per target leaf A.  The particles of every leaf in A's P2P
// list (A itself included) form one stream, staged into LDS in windows of up
// to SRC particles -- FP32 offsets from A's centre in the mixed form, absolute
// FP64 positions in the FP64 form.  Consecutive lanes load consecutive slots,
// each finding its particle from the list entry that holds the slot (a binary
// search over the chunk's stream positions, kept in LDS).
//
// Lanes = (sink, phase), lane = ti * nph + ph: LP = 64 / nph sinks at a time,
// phase ph taking window slots ph, ph + nph, ...  The sinks of A are taken 64
// at a time ("super passes"); within one, `passes` = ceil(ns / LP) passes over
// each staged window cover its ns sinks, LP chosen per leaf so that few lanes
// idle (a leaf of 40 runs 5 passes of 8 sinks x 8 phases rather than one pass
// with 24 of 64 lanes idle).  With one pass a lane accumulates its phase for
// the whole stream and the phases are summed at the end; with several, the
// phases of a pass are summed after every window (DPP within the group of nph
// lanes) and kept by the lane of phase p, the home lane of sink p * LP + ti.
// A window is padded to a multiple of UNROLL*nph with massless sources far
// away, so every lane runs the same number of unrolled blocks with no bounds
// test.  FP32 partial sums are added into FP64 accumulators after every block
// of UNROLL sources.
#define P2P_WAVES 4
#define P2P_UNROLL 8
#define P2P_MAXPH 16  // at most 16 phases, so a window pads to a multiple of 128

template <bool MIXED>
struct P2PTypes;
template <>
struct P2PTypes<true> {
  typedef float R;
  typedef float4 R4;
  static constexpr int SRC = 384;  // multiple of P2P_UNROLL * P2P_MAXPH
  __device__ static R4 far() { return make_float4(1e15f, 1e15f, 1e15f, 0.f); }
};
template <>
struct P2PTypes<false> {
  typedef double R;
  typedef double4 R4;
  static constexpr int SRC = 256;
  __device__ static R4 far() { return make_double4(1e150, 1e150, 1e150, 0.0); }
};

// One block of UNROLL sources of one phase (stride NPH between them).  For
// the Wendland kernel a block in which no pair of the whole wavefront lies
// inside the kernel radius (the common case: such pairs are a tiny fraction)
// takes the -1/r form without a per-pair test; otherwise every pair goes
// through PairKernel, whose outside branch is the same expressions, so the
// sums are the same either way.
template <typename R, typename R4, int KERNEL, bool SELF, int NPH>
__device__ __forceinline__ void p2p_block(const R4 *src, int f0, int self_idx, R xi, R yi, R zi,
                                          R eps2, R inv_eps, R inv_eps3, R &sx, R &sy, R &sz,
                                          R &sp) {
  if (KERNEL == 0) {
    R dx[P2P_UNROLL], dy[P2P_UNROLL], dz[P2P_UNROLL], r2[P2P_UNROLL], mj[P2P_UNROLL];
    {
      R4 svs[P2P_UNROLL];  // the block's sources, read before any use
#pragma unroll
      for (int u = 0; u < P2P_UNROLL; ++u) svs[u] = src[f0 + u * NPH];
#pragma unroll
      for (int u = 0; u < P2P_UNROLL; ++u) {
        dx[u] = svs[u].x - xi;
        dy[u] = svs[u].y - yi;
        dz[u] = svs[u].z - zi;
        r2[u] = fma(dx[u], dx[u], fma(dy[u], dy[u], dz[u] * dz[u]));
        mj[u] = svs[u].w;
        if (SELF) {
          const bool self = f0 + u * NPH == self_idx;
          r2[u] = self ? R(1) : r2[u];
          mj[u] = self ? R(0) : mj[u];
        }
      }
    }
    R rmin = r2[0];
#pragma unroll
    for (int u = 1; u < P2P_UNROLL; ++u) rmin = fmin(rmin, r2[u]);
    if (__ballot(rmin < eps2) == 0ull) {
#pragma unroll
      for (int u = 0; u < P2P_UNROLL; ++u) {
        const R rinv = fast_rsqrt<R>(r2[u]);
        const R t = mj[u] * rinv;
        const R mg = t * (rinv * rinv);
        sx = fma(mg, dx[u], sx);
        sy = fma(mg, dy[u], sy);
        sz = fma(mg, dz[u], sz);
        sp += t;
      }
      return;
    }
    // a pair of the wavefront lies inside the radius: every pair of the block
    // through PairKernel, on the differences already formed
#pragma unroll
    for (int u = 0; u < P2P_UNROLL; ++u) {
      R mg, tp;
      PairKernel<R, KERNEL>::eval(r2[u], mj[u], eps2, inv_eps, inv_eps3, mg, tp);
      sx = fma(mg, dx[u], sx);
      sy = fma(mg, dy[u], sy);
      sz = fma(mg, dz[u], sz);
      sp += tp;
    }
    return;
  }
  // Plummer: every pair through PairKernel
  R4 svs[P2P_UNROLL];
#pragma unroll
  for (int u = 0; u < P2P_UNROLL; ++u) svs[u] = src[f0 + u * NPH];
#pragma unroll
  for (int u = 0; u < P2P_UNROLL; ++u) {
    const R4 sv = svs[u];
    const R dx = sv.x - xi, dy = sv.y - yi, dz = sv.z - zi;
    R r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    R mj = sv.w;
    if (SELF) {
      const bool self = f0 + u * NPH == self_idx;
      r2 = self ? R(1) : r2;
      mj = self ? R(0) : mj;
    }
    R mg, tp;
    PairKernel<R, KERNEL>::eval(r2, mj, eps2, inv_eps, inv_eps3, mg, tp);
    sx = fma(mg, dx, sx);
    sy = fma(mg, dy, sy);
    sz = fma(mg, dz, sz);
    sp += tp;
  }
}

// One phase of one staged window (Wr slots, a multiple of UNROLL * NPH) for
// one sink, added into (bx, by, bz, bp).
template <typename R, typename R4, int KERNEL, bool SELF, int NPH>
__device__ __forceinline__ void p2p_window(const R4 *src, int ph, int Wr, int self_idx, R xi,
                                           R yi, R zi, R eps2, R inv_eps, R inv_eps3, double &bx,
                                           double &by, double &bz, double &bp) {
  constexpr int B = P2P_UNROLL * NPH;  // slots per block of all phases
  int f0 = ph;
  // two blocks per update of the FP64 sums, then the odd block if any
  for (; f0 + B < Wr; f0 += 2 * B) {
    R sx = 0, sy = 0, sz = 0, sp = 0;
    p2p_block<R, R4, KERNEL, SELF, NPH>(src, f0, self_idx, xi, yi, zi, eps2, inv_eps, inv_eps3,
                                        sx, sy, sz, sp);
    p2p_block<R, R4, KERNEL, SELF, NPH>(src, f0 + B, self_idx, xi, yi, zi, eps2, inv_eps,
                                        inv_eps3, sx, sy, sz, sp);
    bx += (double)sx;
    by += (double)sy;
    bz += (double)sz;
    bp -= (double)sp;
  }
  if (f0 < Wr) {
    R sx = 0, sy = 0, sz = 0, sp = 0;
    p2p_block<R, R4, KERNEL, SELF, NPH>(src, f0, self_idx, xi, yi, zi, eps2, inv_eps, inv_eps3,
                                        sx, sy, sz, sp);
    bx += (double)sx;
    by += (double)sy;
    bz += (double)sz;
    bp -= (double)sp;
  }
}

template <typename R, typename R4, int KERNEL, bool SELF>
__device__ __forceinline__ void p2p_window_any(int nph, const R4 *src, int ph, int Wr,
                                               int self_idx, R xi, R yi, R zi, R eps2, R inv_eps,
                                               R inv_eps3, double &bx, double &by, double &bz,
                                               double &bp) {
  switch (nph) {
    case 1:
      p2p_window<R, R4, KERNEL, SELF, 1>(src, ph, Wr, self_idx, xi, yi, zi, eps2, inv_eps,
                                         inv_eps3, bx, by, bz, bp);
      break;
    case 2:
      p2p_window<R, R4, KERNEL, SELF, 2>(src, ph, Wr, self_idx, xi, yi, zi, eps2, inv_eps,
                                         inv_eps3, bx, by, bz, bp);
      break;
    case 4:
      p2p_window<R, R4, KERNEL, SELF, 4>(src, ph, Wr, self_idx, xi, yi, zi, eps2, inv_eps,
                                         inv_eps3, bx, by, bz, bp);
      break;
    case 8:
      p2p_window<R, R4, KERNEL, SELF, 8>(src, ph, Wr, self_idx, xi, yi, zi, eps2, inv_eps,
                                         inv_eps3, bx, by, bz, bp);
      break;
    default:
      p2p_window<R, R4, KERNEL, SELF, 16>(src, ph, Wr, self_idx, xi, yi, zi, eps2, inv_eps,
                                          inv_eps3, bx, by, bz, bp);
      break;
  }
}

// Sum over each aligned group of nph consecutive lanes (nph = 1, 2, 4, 8, 16),
// every lane of a group ending with the same value: quad swaps (lane ^ 1,
// lane ^ 2), then the mirror within 8 and within 16 lanes, each pairing a lane
// with one of the other half whose partial is already the other half's sum.
// All lanes must be active.
__device__ __forceinline__ double group_sum(double v, int nph) {
  if (nph > 1) v += dpp_f<0xB1>(v);   // quad_perm [1,0,3,2]
  if (nph > 2) v += dpp_f<0x4E>(v);   // quad_perm [2,3,0,1]
  if (nph > 4) v += dpp_f<0x141>(v);  // row_half_mirror
  if (nph > 8) v += dpp_f<0x140>(v);  // row_mirror
  return v;
}

// log2 of the sinks per pass for a super pass of ns sinks: the fewest
// lane-slots ceil(ns / LP) * LP, weighted by the cost of the per-window phase
// sums when there is more than one pass; ties go to the larger LP.
__device__ __forceinline__ int p2p_lanes_log2(int ns) {
  int best_lg = 6, best = 1 << 30;
  for (int lg = 6; lg >= 2; --lg) {
    const int LP = 1 << lg, nph = 64 >> lg;
    const int passes = (ns + LP - 1) >> lg;
    const int ovh = passes > 1 ? (nph == 16 ? 8 : nph == 8 ? 3 : nph == 4 ? 1 : 0) : 0;
    const int cost = passes * LP * (64 + ovh);
    if (cost < best) {
      best = cost;
      best_lg = lg;
    }
  }
  return best_lg;
}

// SELF: exclude the self pair by its stream position (needed when eps = 0);
// otherwise the self pair is evaluated -- its acceleration term is exactly
// zero (dx = 0) -- and its potential term, reproduced bit for bit, is taken
// off once per sink.
template <bool MIXED, int KERNEL, bool SELF>
__global__ __launch_bounds__(P2P_WAVES * 64, MIXED ? 4 : 2) void k_p2p(DevTree t, int n_nodes, double eps) {
  typedef typename P2PTypes<MIXED>::R R;
  typedef typename P2PTypes<MIXED>::R4 R4;
  constexpr int SRC = P2PTypes<MIXED>::SRC;
  static_assert(SRC % (P2P_UNROLL * P2P_MAXPH) == 0, "window must hold its padding");
  __shared__ R4 src_all[P2P_WAVES][SRC];
  __shared__ int3 leaf_all[P2P_WAVES][64];  // per list entry of a chunk: stream position, size, first particle
  __shared__ R sink_all[P2P_WAVES][3][64];  // home sink position of each lane
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  R4 *src = src_all[w];
  int3 *lf = leaf_all[w];
  R(*sk)[64] = sink_all[w];
  // the target leaf and all that is read from it are the same in every lane:
  // kept in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(xcd_block<32>(blockIdx.x, gridDim.x) * P2P_WAVES + w);
  const int nwaves = gridDim.x * P2P_WAVES;
  const R eps2 = (R)(eps * eps);
  const R inv_eps = eps > 0 ? (R)(1.0 / eps) : R(0);
  const R inv_eps3 = eps > 0 ? (R)(1.0 / (eps * eps * eps)) : R(0);
  const int64_t cap = t.cap_n;
  n_nodes = node_count(t, n_nodes);
  for (int A = wave; A < n_nodes; A += nwaves) {
    if (t.nnchild[A] != 0 || skipped(t, A)) continue;
    const int bA = t.nbeg[A], nA = t.nend[A] - bA;
    if (!has_sink(t, A, bA, nA)) continue;
    const double4 gA = t.ngeo[A];
    const int off = t.p2p_off[A], cnt = t.p2p_cnt[A];
    for (int tb = 0; tb < nA; tb += 64) {
      const int ns = min(64, nA - tb);
      const int lg = p2p_lanes_log2(ns);
      const int LP = 1 << lg;                  // sinks per pass
      const int nph = 64 >> lg;                // phases
      const int passes = (ns + LP - 1) >> lg;
      const int ti = lane >> (6 - lg), ph = lane & (nph - 1);
      const int blk = P2P_UNROLL * nph;        // slots per unrolled block of all phases
      // home sink of this lane: with one pass sink ti (summed at the end,
      // written by phase 0), else sink ph * LP + ti
      const int hs = passes > 1 ? ph * LP + ti : ti;
      const bool hv = hs < ns && (passes > 1 || ph == 0);
      const int gi = bA + tb + (hs < ns ? hs : 0);
      // home sink positions, kept in LDS across the windows
      if (MIXED) {
        sk[0][lane] = (R)(t.sx[gi] - gA.x);
        sk[1][lane] = (R)(t.sy[gi] - gA.y);
        sk[2][lane] = (R)(t.sz[gi] - gA.z);
      } else {
        sk[0][lane] = t.sx[gi];
        sk[1][lane] = t.sy[gi];
        sk[2][lane] = t.sz[gi];
      }
      double ax = 0, ay = 0, az = 0, pp = 0;
      for (int qb = 0; qb < cnt; qb += 64) {
        const int q = qb + lane;
        const bool vq = q < cnt;
        const int B = vq ? t.p2p_src[off + q] : A;
        const int bB = t.nbeg[B];
        const int nb = vq ? t.nend[B] - bB : 0;
        int total;
        const int pos = wave_excl_scan_int(nb, &total);  // lanes past cnt hold pos = total
        total = __builtin_amdgcn_readfirstlane(total);
        const unsigned long long selfm = __ballot(vq && B == A);
        const int self_lane = selfm ? (int)__ffsll((long long)selfm) - 1 : 0;
        const int self_start =
            __builtin_amdgcn_readfirstlane(selfm ? __shfl(pos, self_lane, 64) : -(1 << 30));
        lf[lane] = make_int3(pos, nb, bB);  // kept in LDS across the windows
        __builtin_amdgcn_wave_barrier();
        for (int w0 = 0; w0 < total; w0 += SRC) {
          const int W = min(SRC, total - w0);
          const int Wr = (W + blk - 1) / blk * blk;
          // consecutive lanes stage consecutive slots, two per lane at a
          // time; a slot's particle comes from the list entry holding its
          // stream position, the last entry whose position is not beyond it
          // (binary search over the chunk's entries)
          for (int j0 = 0; j0 < Wr; j0 += 128) {
            const int ja = j0 + lane, jb = ja + 64;
            const int sa = w0 + ja, sb = w0 + jb;
            int ea = 0, eb = 0;
#pragma unroll
            for (int st = 32; st > 0; st >>= 1) {
              if (lf[ea + st].x <= sa) ea += st;
              if (lf[eb + st].x <= sb) eb += st;
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int j = h ? jb : ja;
              if (j < Wr) {
                R4 v = P2PTypes<MIXED>::far();
                if (j < W) {
                  const int3 en = lf[h ? eb : ea];
                  const int k = en.z + (w0 + j - en.x);
                  if (MIXED) {
                    v.x = (R)(t.sx[k] - gA.x);
                    v.y = (R)(t.sy[k] - gA.y);
                    v.z = (R)(t.sz[k] - gA.z);
                    v.w = t.sm32[k];
                  } else {
                    v.x = t.sx[k];
                    v.y = t.sy[k];
                    v.z = t.sz[k];
                    v.w = t.sm[k];
                  }
                }
                src[j] = v;
              }
            }
          }
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
          if (passes == 1) {
            p2p_window_any<R, R4, KERNEL, SELF>(nph, src, ph, Wr, self_start + tb + ti - w0,
                                                sk[0][lane], sk[1][lane], sk[2][lane], eps2,
                                                inv_eps, inv_eps3, ax, ay, az, pp);
          } else {
            for (int p = 0; p < passes; ++p) {
              const int from = ti * nph + p;  // home lane of sink p * LP + ti
              const R xi = sk[0][from], yi = sk[1][from], zi = sk[2][from];
              double bx = 0, by = 0, bz = 0, bp = 0;
              p2p_window_any<R, R4, KERNEL, SELF>(nph, src, ph, Wr,
                                                  self_start + tb + p * LP + ti - w0, xi, yi, zi,
                                                  eps2, inv_eps, inv_eps3, bx, by, bz, bp);
              bx = group_sum(bx, nph);
              by = group_sum(by, nph);
              bz = group_sum(bz, nph);
              bp = group_sum(bp, nph);
              if (ph == p) {
                ax += bx;
                ay += by;
                az += bz;
                pp += bp;
              }
            }
          }
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        }
      }
      if (passes == 1) {
        ax = group_sum(ax, nph);
        ay = group_sum(ay, nph);
        az = group_sum(az, nph);
        pp = group_sum(pp, nph);
      }
      if (!SELF) {  // the self pair's potential term, as the loop computed it
        R mg0, t0;
        PairKernel<R, KERNEL>::eval(R(0), MIXED ? (R)t.sm32[gi] : (R)t.sm[gi], eps2, inv_eps,
                                    inv_eps3, mg0, t0);
        pp += (double)t0;
      }
      if (hv) {
        t.near[gi] = ax;
        t.near[cap + gi] = ay;
        t.near[2 * cap + gi] = az;
        t.near[3 * cap + gi] = pp;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Cells of level l for a launch with per_cell threads per cell: exact, or
// (e.dev) an estimated grid and bounds read on the device.
static void level_launch(const EvalArgs &e, int l, int per_cell, int &blocks, int &a0, int &a1) {
  const int ls = e.lvl_start_host[l], le = e.lvl_start_host[l + 1];
  const int cnt = le - ls;
  if (!e.dev) {
    blocks = cnt > 0 ? (per_cell * cnt + FMM_BLOCK - 1) / FMM_BLOCK : 0;
    a0 = ls;
    a1 = le;
  } else if (e.exact) {
    blocks = cnt > 0 ? (per_cell * cnt + FMM_BLOCK - 1) / FMM_BLOCK : 0;
    a0 = -1 - l;
    a1 = 0;
  } else {
    blocks = (per_cell * (cnt + cnt / 4 + 32) + FMM_BLOCK - 1) / FMM_BLOCK;
    a0 = -1 - l;
    a1 = 0;
  }
}

// Upward pass: P2M and M2M (far-field cell kernels: 8 lanes per cell).
template <typename T, int P, int KERNEL>
static void run_upward(const DevTree &t, const EvalArgs &e, hipStream_t s) {
  const int nn = e.n_nodes;
  const int ga = e.dev ? nn + nn / 4 + 64 : nn;
  const int narg = e.dev ? -1 : nn;
  const bool harm = KERNEL == 0;  // folded moments feed the harmonic M2L
  hipLaunchKernelGGL((k_p2m<T, P>), dim3((8 * ga + FMM_BLOCK - 1) / FMM_BLOCK), dim3(FMM_BLOCK), 0,
                     s, t, narg, harm);
  if (nn <= SMALL_NODES && e.depth > 0) {
    hipLaunchKernelGGL((k_m2m_small<T, P>), dim3(1), dim3(FMM_BLOCK), 0, s, t, e.depth, harm,
                       e.dev);
  } else {
    for (int l = e.depth - 1; l >= 0; --l) {
      int blocks, a0, a1;
      level_launch(e, l, 8, blocks, a0, a1);
      if (blocks > 0)
        hipLaunchKernelGGL((k_m2m<T, P>), dim3(blocks), dim3(FMM_BLOCK), 0, s, t, a0, a1, harm);
    }
  }
}

// Launch order: P2P goes to the side stream (after the walk and the mass
// gather, by an event) and runs concurrently with M2L and L2L on the main
// stream, which waits for it (second event) before L2P adds the near field.
// P2M and M2M run on the main stream before M2L, unless launch_upward already
// queued them on the side stream beside the walk (e.upward_done): then the
// main stream waits for e.up_done instead.
template <typename T, int P, int KERNEL>
static void run_passes(const DevTree &t, const EvalArgs &e, hipStream_t s) {
  const int nn = e.n_nodes;  // exact, or (e.dev) an estimate that sets grid sizes
  const int ga = e.dev && !e.exact ? nn + nn / 4 + 64 : nn;
  const int narg = e.dev ? -1 : nn;  // -1: node count read on the device
  PhaseTimer *tm = e.tm;
  hipEventRecord(e.fork, s);
  hipStreamWaitEvent(e.side, e.fork, 0);
  const int tp = tm ? tm->begin(PH_P2P, e.side) : -1;
  if (e.eps > 0)
    hipLaunchKernelGGL((k_p2p<(sizeof(T) == 4), KERNEL, false>),
                       dim3((ga + P2P_WAVES - 1) / P2P_WAVES), dim3(P2P_WAVES * 64), 0, e.side,
                       t, narg, e.eps);
  else
    hipLaunchKernelGGL((k_p2p<(sizeof(T) == 4), KERNEL, true>),
                       dim3((ga + P2P_WAVES - 1) / P2P_WAVES), dim3(P2P_WAVES * 64), 0, e.side,
                       t, narg, e.eps);
  if (tm) tm->end(tp, e.side);
  hipEventRecord(e.join, e.side);
  if (e.upward_done)
    hipStreamWaitEvent(s, e.up_done, 0);  // P2M / M2M ran beside the walk
  else
    run_upward<T, P, KERNEL>(t, e, s);
  const bool small = nn <= SMALL_NODES;
  const int wave_blocks = (ga + 3) / 4;
  if (tm) {
    tm->stop(s);
    tm->start(PH_M2L, s);
  }
  hipLaunchKernelGGL((k_m2l<T, P, KERNEL>), dim3(wave_blocks), dim3(FMM_BLOCK), 0, s, t, narg,
                     e.eps);
  if (tm) {
    tm->stop(s);
    tm->start(PH_DOWN, s);
  }
  if (small && e.depth > 0) {
    hipLaunchKernelGGL((k_l2l_small<T, P>), dim3(1), dim3(FMM_BLOCK), 0, s, t, e.depth, e.dev);
  } else {
    for (int l = 1; l <= e.depth; ++l) {
      int blocks, a0, a1;
      level_launch(e, l, 1, blocks, a0, a1);
      if (blocks > 0)
        hipLaunchKernelGGL((k_l2l<T, P>), dim3(blocks), dim3(FMM_BLOCK), 0, s, t, a0, a1);
    }
  }
  hipStreamWaitEvent(s, e.join, 0);
  hipLaunchKernelGGL((k_l2p<T, P>), dim3((e.n + FMM_BLOCK - 1) / FMM_BLOCK), dim3(FMM_BLOCK), 0,
                     s, t, e.n, e.dev, 1.0);
  if (tm) tm->stop(s);
}

template <typename T, int KERNEL>
static bool dispatch_order(const DevTree &t, const EvalArgs &e, hipStream_t s) {
  switch (e.p) {
    case 1: run_passes<T, 1, KERNEL>(t, e, s); return true;
    case 2: run_passes<T, 2, KERNEL>(t, e, s); return true;
    case 3: run_passes<T, 3, KERNEL>(t, e, s); return true;
    case 4: run_passes<T, 4, KERNEL>(t, e, s); return true;
    case 5: run_passes<T, 5, KERNEL>(t, e, s); return true;
    case 6: run_passes<T, 6, KERNEL>(t, e, s); return true;
    default: return false;
  }
}

bool eval_order_supported(int p) { return p >= 1 && p <= 6; }

template <typename T, int KERNEL>
static bool dispatch_upward(const DevTree &t, const EvalArgs &e, hipStream_t s) {
  switch (e.p) {
    case 1: run_upward<T, 1, KERNEL>(t, e, s); return true;
    case 2: run_upward<T, 2, KERNEL>(t, e, s); return true;
    case 3: run_upward<T, 3, KERNEL>(t, e, s); return true;
    case 4: run_upward<T, 4, KERNEL>(t, e, s); return true;
    case 5: run_upward<T, 5, KERNEL>(t, e, s); return true;
    case 6: run_upward<T, 6, KERNEL>(t, e, s); return true;
    default: return false;
  }
}

hipError_t launch_upward(const DevTree &t, const EvalArgs &e, hipStream_t s) {
  if (e.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_mass, dim3((e.n + FMM_BLOCK - 1) / FMM_BLOCK), dim3(FMM_BLOCK), 0, s,
                     t, e.n);
  bool ok;
  if (e.mixed)
    ok = e.kernel == 1 ? dispatch_upward<float, 1>(t, e, s) : dispatch_upward<float, 0>(t, e, s);
  else
    ok = e.kernel == 1 ? dispatch_upward<double, 1>(t, e, s) : dispatch_upward<double, 0>(t, e, s);
  if (!ok) return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_evaluate(const DevTree &t, const EvalArgs &e, hipStream_t s) {
  if (e.n <= 0) return hipSuccess;
  if (e.tm) e.tm->start(PH_UP, s);
  if (!e.upward_done)
    hipLaunchKernelGGL(k_gather_mass, dim3((e.n + FMM_BLOCK - 1) / FMM_BLOCK), dim3(FMM_BLOCK), 0,
                       s, t, e.n);
  bool ok;
  if (e.mixed)
    ok = e.kernel == 1 ? dispatch_order<float, 1>(t, e, s) : dispatch_order<float, 0>(t, e, s);
  else
    ok = e.kernel == 1 ? dispatch_order<double, 1>(t, e, s) : dispatch_order<double, 0>(t, e, s);
  if (!ok) return hipErrorInvalidValue;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Vector-source pass on the tree of the last build (one system): sources
// m_j v_j, output u = +gradient of their potential (the derivative of the
// accelerations along the displacement field v) and that potential.  All on
// stream s: gather, dipole P2M, M2M, M2L, L2L, near field (grad.hip), L2P.
template <typename T, int P, int KERNEL>
static void run_dipole(const DevTree &t, const EvalArgs &e, const double *vec, double *dv,
                       hipStream_t s) {
  const int nn = e.n_nodes;
  const bool harm = KERNEL == 0;
  hipLaunchKernelGGL(k_gather_dip, dim3((e.n + FMM_BLOCK - 1) / FMM_BLOCK), dim3(FMM_BLOCK), 0, s,
                     t, e.n, vec, dv);
  hipLaunchKernelGGL((k_p2m_dip<T, P>), dim3((8 * nn + FMM_BLOCK - 1) / FMM_BLOCK),
                     dim3(FMM_BLOCK), 0, s, t, nn, (const double *)dv, harm);
  if (nn <= SMALL_NODES && e.depth > 0) {
    hipLaunchKernelGGL((k_m2m_small<T, P>), dim3(1), dim3(FMM_BLOCK), 0, s, t, e.depth, harm,
                       false);
  } else {
    for (int l = e.depth - 1; l >= 0; --l) {
      int blocks, a0, a1;
      level_launch(e, l, 8, blocks, a0, a1);
      if (blocks > 0)
        hipLaunchKernelGGL((k_m2m<T, P>), dim3(blocks), dim3(FMM_BLOCK), 0, s, t, a0, a1, harm);
    }
  }
  hipLaunchKernelGGL((k_m2l<T, P, KERNEL>), dim3((nn + 3) / 4), dim3(FMM_BLOCK), 0, s, t, nn,
                     e.eps);
  if (nn <= SMALL_NODES && e.depth > 0) {
    hipLaunchKernelGGL((k_l2l_small<T, P>), dim3(1), dim3(FMM_BLOCK), 0, s, t, e.depth, false);
  } else {
    for (int l = 1; l <= e.depth; ++l) {
      int blocks, a0, a1;
      level_launch(e, l, 1, blocks, a0, a1);
      if (blocks > 0)
        hipLaunchKernelGGL((k_l2l<T, P>), dim3(blocks), dim3(FMM_BLOCK), 0, s, t, a0, a1);
    }
  }
  launch_p2p_dipole(t, nn, e.kernel, sizeof(T) == 4, e.eps, dv, s);
  hipLaunchKernelGGL((k_l2p<T, P>), dim3((e.n + FMM_BLOCK - 1) / FMM_BLOCK), dim3(FMM_BLOCK), 0,
                     s, t, e.n, false, -1.0);
}

template <typename T, int KERNEL>
static bool dispatch_dipole(const DevTree &t, const EvalArgs &e, const double *vec, double *dv,
                            hipStream_t s) {
  switch (e.p) {
    case 1: run_dipole<T, 1, KERNEL>(t, e, vec, dv, s); return true;
    case 2: run_dipole<T, 2, KERNEL>(t, e, vec, dv, s); return true;
    case 3: run_dipole<T, 3, KERNEL>(t, e, vec, dv, s); return true;
    case 4: run_dipole<T, 4, KERNEL>(t, e, vec, dv, s); return true;
    case 5: run_dipole<T, 5, KERNEL>(t, e, vec, dv, s); return true;
    case 6: run_dipole<T, 6, KERNEL>(t, e, vec, dv, s); return true;
    default: return false;
  }
}

hipError_t launch_dipole(const DevTree &t, const EvalArgs &e, const double *vec, double *dv,
                         hipStream_t s) {
  if (e.n <= 0) return hipSuccess;
  bool ok;
  if (e.mixed)
    ok = e.kernel == 1 ? dispatch_dipole<float, 1>(t, e, vec, dv, s)
                       : dispatch_dipole<float, 0>(t, e, vec, dv, s);
  else
    ok = e.kernel == 1 ? dispatch_dipole<double, 1>(t, e, vec, dv, s)
                       : dispatch_dipole<double, 0>(t, e, vec, dv, s);
  if (!ok) return hipErrorInvalidValue;
  return hipGetLastError();
}
