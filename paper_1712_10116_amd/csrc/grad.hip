// Force gradient d a_i / d x_i (the tidal tensor) of every active particle,
// the quantity the forward fourth-order integrator of Sec. 4.1 needs from the
// FMM, computed on the tree, lists and local expansions of the evaluation
// just made: minus the Hessian of the leaf's local expansion, plus for every
// particle of every leaf in the sink leaf's P2P list the derivative of
// m g(r) d (d = x_j - x_i) with respect to x_i, -m (g I + (dg/dr)/r d d^T).
// Output SoA, 6 rows of n: xx, yy, zz, xy, xz, yz, in active order.
//
// Both parts run in the evaluation's precision (the near part's pair terms
// on offsets from the sink leaf's centre, summed into FP64 per source leaf).
#include "common.h"
#include "expansion.h"

namespace {

constexpr int CA[6] = {0, 1, 2, 0, 0, 1}, CB[6] = {0, 1, 2, 1, 2, 2};

// g = psi'(r)/r and h = (dg/dr)/r of the pair kernel.  Wendland C2 (Eq. 8):
// inside the radius g = (21u^5 - 90u^4 + 140u^3 - 84u^2 + 14)/eps^3 and h =
// (105u^3 - 360u^2 + 420u - 168)/eps^5 (u = r/eps), outside 1/r^3 and
// -3/r^5; Plummer: s^(-3/2) and -3 s^(-5/2), s = r^2 + eps^2.
template <typename R, int KERNEL>
__device__ __forceinline__ void pair_gh(R r2, R eps, R ie, R &g, R &h) {
  if (KERNEL == 1) {
    const R rs = fast_rsqrt<R>(r2 + eps * eps), is = rs * rs;
    g = is * rs;
    h = R(-3) * g * is;
  } else {
    const R ir = fast_rsqrt<R>(r2);
    if (r2 >= eps * eps) {
      const R ir2 = ir * ir;
      g = ir2 * ir;
      h = R(-3) * g * ir2;
    } else {
      const R u = r2 > R(0) ? r2 * ir * ie : R(0), ie3 = ie * ie * ie;
      g = ((((R(21) * u - R(90)) * u + R(140)) * u - R(84)) * u * u + R(14)) * ie3;
      h = (((R(105) * u - R(360)) * u + R(420)) * u - R(168)) * ie3 * ie * ie;
    }
  }
}

// A staged source: its offset from the sink leaf's centre and its mass, in R.
template <typename R>
struct alignas(4 * sizeof(R)) SrcR {
  R x, y, z, m;
};

// near part: one wavefront per sink leaf, lanes over its sinks (and, for
// leaves of at most 32, over 2-16 phases of the sources), each source leaf
// staged through LDS 64 particles at a time as offsets from the sink leaf's
// centre in R (FP32 in the mixed form: cell-local offsets, as in the forces'
// P2P); pair terms in R, summed in R over one source leaf and then into FP64.
// Per pair: m h d (3 products) and six FMAs of it with d for the h d d^T
// part; the g I part is one sum of m g per source leaf.  The self pair (d = 0)
// is masked by a select, so an infinite g or h there never reaches a sum.
// Written in sorted order to stage (6 rows of stride cap_n); k_l2p_grad adds
// the far part and writes each particle's tensor once in active order.
template <typename R, int KERNEL>
__global__ __launch_bounds__(FMM_BLOCK) void k_p2p_grad(DevTree t, int n_nodes, double eps,
                                                        double *__restrict__ stage) {
  const int lane = threadIdx.x & 63;
  // neighbouring leaves, which share most of their sources, on one XCD
  const int wave =
      __builtin_amdgcn_readfirstlane((xcd_block<32>(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) >> 6);
  const int nwaves = (gridDim.x * blockDim.x) >> 6;
  const R reps = (R)eps, ie = eps > 0 ? (R)(1.0 / eps) : R(0);
  __shared__ SrcR<R> src_lds[FMM_BLOCK / 64][64];
  SrcR<R> *st = src_lds[threadIdx.x >> 6];
  for (int A = wave; A < n_nodes; A += nwaves) {
    if (t.nnchild[A] != 0) continue;
    const int bA = t.nbeg[A], nA = t.nend[A] - bA;
    const int loff = t.p2p_off[A], cnt = t.p2p_cnt[A];
    const double4 gA = t.ngeo[A];
    for (int tb = 0; tb < nA; tb += 64) {
      // lanes = (sink, phase): nph phases share each sink and take every
      // nph-th source, so a leaf of fewer than 64 sinks still fills the wave
      const int ns = min(64, nA - tb);
      const int nph = ns <= 4 ? 16 : ns <= 8 ? 8 : ns <= 16 ? 4 : ns <= 32 ? 2 : 1;
      const int ti = lane / nph, ph = lane % nph;
      const bool valid = ti < ns;
      const int i = bA + tb + (valid ? ti : 0);
      // the sink's offset, formed exactly as a staged source's
      const R xi = (R)(t.sx[i] - gA.x), yi = (R)(t.sy[i] - gA.y), zi = (R)(t.sz[i] - gA.z);
      double G[6] = {0, 0, 0, 0, 0, 0};
      for (int q = 0; q < cnt; ++q) {
        const int B = t.p2p_src[loff + q];
        const int eB = t.nend[B];
        R Gs[6] = {0, 0, 0, 0, 0, 0};
        R Gg = 0;
        for (int jb = t.nbeg[B]; jb < eB; jb += 64) {
          // up to 64 sources of leaf B staged in LDS by the wave's lanes
          const int nj = min(64, eB - jb);
          SrcR<R> e{R(0), R(0), R(0), R(0)};
          if (lane < nj)
            e = SrcR<R>{(R)(t.sx[jb + lane] - gA.x), (R)(t.sy[jb + lane] - gA.y),
                        (R)(t.sz[jb + lane] - gA.z), (R)t.sm[jb + lane]};
          st[lane] = e;
          __builtin_amdgcn_wave_barrier();
          // every lane takes the same number of steps: slot ph + k, k = 0, nph,
          // ..., stays below 64 (nph divides 64); slots past nj hold zeros
          const int si = i - jb - ph, lim = nj - ph;
          for (int k = 0; k < nj; k += nph) {
            const SrcR<R> sv = st[ph + k];
            const R dx = sv.x - xi, dy = sv.y - yi, dz = sv.z - zi;
            const R r2 = fma(dz, dz, fma(dy, dy, dx * dx));
            R g, h;
            pair_gh<R, KERNEL>(r2, reps, ie, g, h);
            const bool skip = k == si || k >= lim;
            const R mg = skip ? R(0) : sv.m * g;
            const R mh = skip ? R(0) : sv.m * h;
            const R hx = mh * dx, hy = mh * dy, hz = mh * dz;
            Gg += mg;
            Gs[0] = fma(-hx, dx, Gs[0]);
            Gs[1] = fma(-hy, dy, Gs[1]);
            Gs[2] = fma(-hz, dz, Gs[2]);
            Gs[3] = fma(-hx, dy, Gs[3]);
            Gs[4] = fma(-hx, dz, Gs[4]);
            Gs[5] = fma(-hy, dz, Gs[5]);
          }
          __builtin_amdgcn_wave_barrier();
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) G[c] += (double)(Gs[c] - Gg);
#pragma unroll
        for (int c = 3; c < 6; ++c) G[c] += (double)Gs[c];
      }
      // the phases of a sink are consecutive lanes: fold them onto phase 0
      for (int o = nph >> 1; o > 0; o >>= 1)
#pragma unroll
        for (int c = 0; c < 6; ++c) G[c] += __shfl_xor(G[c], o, 64);
      if (valid && ph == 0) {
        const int64_t cap = t.cap_n;
#pragma unroll
        for (int c = 0; c < 6; ++c) stage[c * cap + i] = G[c];
      }
    }
  }
}

// minus the Hessian of the leaf's local expansion (coefficients scaled by
// h^|n|, so the second derivatives carry 1/h^2) added to the near part staged
// in sorted order, written to grad in active order (zero for p = 1: the
// Hessian of a degree-1 expansion vanishes)
template <typename T, int P>
__global__ __launch_bounds__(FMM_BLOCK) void k_l2p_grad(DevTree t, int n,
                                                        const double *__restrict__ stage,
                                                        double *__restrict__ grad, int64_t nq,
                                                        int32_t off) {
  constexpr MI<P> mi{};
  constexpr int K = MI<P>::K;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int leaf = t.leaf_of[j];
  const double4 g = t.ngeo[leaf];
  const double ih = 1.0 / g.w;
  T mono[K], Lt[K];
  monomials<T, P>((T)((t.sx[j] - g.x) * ih), (T)((t.sy[j] - g.y) * ih),
                  (T)((t.sz[j] - g.z) * ih), mono);
  const T *row = (const T *)t.L + (size_t)leaf * t.kmax;
#pragma unroll
  for (int k = 0; k < K; ++k) Lt[k] = row[k];
  T H[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (mi.deg[k] + 2 > P) continue;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const int a = mi.x[k] + (CA[c] == 0) + (CB[c] == 0);
      const int b = mi.y[k] + (CA[c] == 1) + (CB[c] == 1);
      const int e = mi.z[k] + (CA[c] == 2) + (CB[c] == 2);
      H[c] = fma(Lt[mi.at(a, b, e)], mono[k], H[c]);
    }
  }
  const int64_t k = t.slot[j] - off, cap = t.cap_n;
  const double s2 = ih * ih;
#pragma unroll
  for (int c = 0; c < 6; ++c) grad[c * nq + k] = stage[c * cap + j] - (double)H[c] * s2;
}

template <typename T, int P>
void launch_l2p_grad(const DevTree &t, int n, const double *stage, double *grad, hipStream_t s) {
  hipLaunchKernelGGL((k_l2p_grad<T, P>), dim3((n + FMM_BLOCK - 1) / FMM_BLOCK), dim3(FMM_BLOCK),
                     0, s, t, n, stage, grad, (int64_t)n, 0);
}

template <typename T, int KERNEL>
bool dispatch_grad(const DevTree &t, int n_nodes, int n, int p, double eps, double *stage,
                   double *grad, hipStream_t s) {
  hipLaunchKernelGGL((k_p2p_grad<T, KERNEL>), dim3((n_nodes + 3) / 4), dim3(FMM_BLOCK), 0, s, t,
                     n_nodes, eps, stage);
  switch (p) {
    case 1: launch_l2p_grad<T, 1>(t, n, stage, grad, s); return true;
    case 2: launch_l2p_grad<T, 2>(t, n, stage, grad, s); return true;
    case 3: launch_l2p_grad<T, 3>(t, n, stage, grad, s); return true;
    case 4: launch_l2p_grad<T, 4>(t, n, stage, grad, s); return true;
    case 5: launch_l2p_grad<T, 5>(t, n, stage, grad, s); return true;
    case 6: launch_l2p_grad<T, 6>(t, n, stage, grad, s); return true;
    default: return false;
  }
}

// Near field of the vector-source pass: for every sink i the sum over the
// particles j of its leaf's P2P partners (j != i) of m_j H(x_i - x_j) v_j,
// H = g I + h d d^T the pair Hessian, and of m_j v_j . grad psi(x_i - x_j)
// = -m_j g (v_j . d), d = x_j - x_i.  Written to near[] in sorted order with
// the sign of an acceleration (minus the field) so that L2P adds the far
// field's gradient the same way.  Layout as k_p2p_grad: one wavefront per
// sink leaf, (sink, phase) lanes, each source leaf staged through LDS 64
// particles at a time (offsets from the sink leaf's centre, mass and vector
// in R), pair terms in R, summed in R over one source leaf and then into FP64.
template <typename R, int KERNEL>
__global__ __launch_bounds__(FMM_BLOCK) void k_p2p_dip(DevTree t, int n_nodes, double eps,
                                                       const double *__restrict__ dv) {
  const int lane = threadIdx.x & 63;
  // neighbouring leaves, which share most of their sources, on one XCD
  const int wave =
      __builtin_amdgcn_readfirstlane((xcd_block<32>(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x) >> 6);
  const int nwaves = (gridDim.x * blockDim.x) >> 6;
  const R reps = (R)eps, ie = eps > 0 ? (R)(1.0 / eps) : R(0);
  const int64_t cap = t.cap_n;
  __shared__ SrcR<R> stage_x[FMM_BLOCK / 64][64];
  __shared__ SrcR<R> stage_v[FMM_BLOCK / 64][64];
  SrcR<R> *sx = stage_x[threadIdx.x >> 6];
  SrcR<R> *sv = stage_v[threadIdx.x >> 6];
  for (int A = wave; A < n_nodes; A += nwaves) {
    if (t.nnchild[A] != 0) continue;
    const int bA = t.nbeg[A], nA = t.nend[A] - bA;
    const int loff = t.p2p_off[A], cnt = t.p2p_cnt[A];
    const double4 gA = t.ngeo[A];
    for (int tb = 0; tb < nA; tb += 64) {
      const int ns = min(64, nA - tb);
      const int nph = ns <= 4 ? 16 : ns <= 8 ? 8 : ns <= 16 ? 4 : ns <= 32 ? 2 : 1;
      const int ti = lane / nph, ph = lane % nph;
      const bool valid = ti < ns;
      const int i = bA + tb + (valid ? ti : 0);
      const R xi = (R)(t.sx[i] - gA.x), yi = (R)(t.sy[i] - gA.y), zi = (R)(t.sz[i] - gA.z);
      double U[4] = {0, 0, 0, 0};
      for (int q = 0; q < cnt; ++q) {
        const int B = t.p2p_src[loff + q];
        const int eB = t.nend[B];
        R Us[4] = {0, 0, 0, 0};
        for (int jb = t.nbeg[B]; jb < eB; jb += 64) {
          const int nj = min(64, eB - jb);
          SrcR<R> ex{R(0), R(0), R(0), R(0)}, ev{R(0), R(0), R(0), R(0)};
          if (lane < nj) {
            const int j = jb + lane;
            ex = SrcR<R>{(R)(t.sx[j] - gA.x), (R)(t.sy[j] - gA.y), (R)(t.sz[j] - gA.z),
                         (R)t.sm[j]};
            ev = SrcR<R>{(R)dv[j], (R)dv[cap + j], (R)dv[2 * cap + j], R(0)};
          }
          sx[lane] = ex;
          sv[lane] = ev;
          __builtin_amdgcn_wave_barrier();
          // same number of steps on every lane, as in k_p2p_grad
          const int si = i - jb - ph, lim = nj - ph;
          for (int k = 0; k < nj; k += nph) {
            const SrcR<R> p = sx[ph + k], v = sv[ph + k];
            const R dx = p.x - xi, dy = p.y - yi, dz = p.z - zi;
            const R r2 = fma(dz, dz, fma(dy, dy, dx * dx));
            R g, h;
            pair_gh<R, KERNEL>(r2, reps, ie, g, h);
            const bool skip = k == si || k >= lim;
            const R mg = skip ? R(0) : p.m * g;
            const R mh = skip ? R(0) : p.m * h;
            const R dvv = fma(dz, v.z, fma(dy, v.y, dx * v.x));
            const R mhd = mh * dvv;
            Us[0] = fma(mg, v.x, fma(mhd, dx, Us[0]));
            Us[1] = fma(mg, v.y, fma(mhd, dy, Us[1]));
            Us[2] = fma(mg, v.z, fma(mhd, dz, Us[2]));
            Us[3] = fma(-mg, dvv, Us[3]);
          }
          __builtin_amdgcn_wave_barrier();
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) U[c] += (double)Us[c];
      }
      for (int o = nph >> 1; o > 0; o >>= 1)
#pragma unroll
        for (int c = 0; c < 4; ++c) U[c] += __shfl_xor(U[c], o, 64);
      if (valid && ph == 0) {
        t.near[i] = -U[0];
        t.near[cap + i] = -U[1];
        t.near[2 * cap + i] = -U[2];
        t.near[3 * cap + i] = U[3];
      }
    }
  }
}

}  // namespace

hipError_t launch_p2p_dipole(const DevTree &t, int n_nodes, int kernel, bool mixed, double eps,
                             const double *dv, hipStream_t s) {
  const dim3 grid((n_nodes + 3) / 4), blk(FMM_BLOCK);
  if (mixed) {
    if (kernel == 1)
      hipLaunchKernelGGL((k_p2p_dip<float, 1>), grid, blk, 0, s, t, n_nodes, eps, dv);
    else
      hipLaunchKernelGGL((k_p2p_dip<float, 0>), grid, blk, 0, s, t, n_nodes, eps, dv);
  } else {
    if (kernel == 1)
      hipLaunchKernelGGL((k_p2p_dip<double, 1>), grid, blk, 0, s, t, n_nodes, eps, dv);
    else
      hipLaunchKernelGGL((k_p2p_dip<double, 0>), grid, blk, 0, s, t, n_nodes, eps, dv);
  }
  return hipGetLastError();
}

// One system's tree (request 0 at slot offset 0), n active particles.
hipError_t launch_force_gradient(const DevTree &t, int n_nodes, int n, int p, int kernel,
                                 bool mixed, double eps, double *stage, double *grad,
                                 hipStream_t s) {
  if (n <= 0) return hipSuccess;
  bool ok;
  if (mixed)
    ok = kernel == 1 ? dispatch_grad<float, 1>(t, n_nodes, n, p, eps, stage, grad, s)
                     : dispatch_grad<float, 0>(t, n_nodes, n, p, eps, stage, grad, s);
  else
    ok = kernel == 1 ? dispatch_grad<double, 1>(t, n_nodes, n, p, eps, stage, grad, s)
                     : dispatch_grad<double, 0>(t, n_nodes, n, p, eps, stage, grad, s);
  if (!ok) return hipErrorInvalidValue;
  return hipGetLastError();
}
