// Force gradient d a_i / d x_i (the tidal tensor) of every active particle,
// the quantity the forward fourth-order integrator of Sec. 4.1 needs from the
// FMM, computed on the tree, lists and local expansions of the evaluation
// just made: minus the Hessian of the leaf's local expansion, plus for every
// particle of every leaf in the sink leaf's P2P list the derivative of
// m g(r) d (d = x_j - x_i) with respect to x_i, -m (g I + (dg/dr)/r d d^T).
// Output SoA, 6 rows of n: xx, yy, zz, xy, xz, yz, in active order.
//
// The near part runs in FP64 in both precisions (one wavefront per sink
// leaf, lanes over its sinks, the sources read in the same order by every
// lane); the far part in the evaluation's precision.
#include "common.h"
#include "expansion.h"

namespace {

constexpr int CA[6] = {0, 1, 2, 0, 0, 1}, CB[6] = {0, 1, 2, 1, 2, 2};

// g = psi'(r)/r and h = (dg/dr)/r of the pair kernel.  Wendland C2 (Eq. 8):
// inside the radius g = (21u^5 - 90u^4 + 140u^3 - 84u^2 + 14)/eps^3 and h =
// (105u^3 - 360u^2 + 420u - 168)/eps^5 (u = r/eps), outside 1/r^3 and
// -3/r^5; Plummer: s^(-3/2) and -3 s^(-5/2), s = r^2 + eps^2.
template <int KERNEL>
__device__ __forceinline__ void pair_gh(double r2, double eps, double &g, double &h) {
  if (KERNEL == 1) {
    const double s = r2 + eps * eps;
    const double is = 1.0 / s, rs = 1.0 / sqrt(s);
    g = is * rs;
    h = -3.0 * g * is;
  } else {
    const double r = sqrt(r2);
    if (r >= eps) {
      const double ir = 1.0 / r, ir2 = ir * ir;
      g = ir2 * ir;
      h = -3.0 * g * ir2;
    } else {
      const double u = r / eps, ie = 1.0 / eps, ie3 = ie * ie * ie;
      g = ((((21.0 * u - 90.0) * u + 140.0) * u - 84.0) * u * u + 14.0) * ie3;
      h = (((105.0 * u - 360.0) * u + 420.0) * u - 168.0) * ie3 * ie * ie;
    }
  }
}

template <int KERNEL>
__global__ __launch_bounds__(FMM_BLOCK) void k_p2p_grad(DevTree t, int n_nodes, double eps,
                                                        double *__restrict__ grad, int64_t nq,
                                                        int32_t off) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int nwaves = (gridDim.x * blockDim.x) >> 6;
  for (int A = wave; A < n_nodes; A += nwaves) {
    if (t.nnchild[A] != 0) continue;
    const int bA = t.nbeg[A], nA = t.nend[A] - bA;
    const int loff = t.p2p_off[A], cnt = t.p2p_cnt[A];
    for (int tb = 0; tb < nA; tb += 64) {
      const bool valid = tb + lane < nA;
      const int i = bA + tb + (valid ? lane : 0);
      const double xi = t.sx[i], yi = t.sy[i], zi = t.sz[i];
      double G[6] = {0, 0, 0, 0, 0, 0};
      for (int q = 0; q < cnt; ++q) {
        const int B = t.p2p_src[loff + q];
        for (int j = t.nbeg[B]; j < t.nend[B]; ++j) {
          if (j == i) continue;
          const double d[3] = {t.sx[j] - xi, t.sy[j] - yi, t.sz[j] - zi};
          const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
          double g, h;
          pair_gh<KERNEL>(r2, eps, g, h);
          const double m = t.sm[j];
#pragma unroll
          for (int c = 0; c < 6; ++c)
            G[c] += m * (-h * d[CA[c]] * d[CB[c]] - (CA[c] == CB[c] ? g : 0.0));
        }
      }
      if (valid) {
        const int64_t k = t.slot[i] - off;
#pragma unroll
        for (int c = 0; c < 6; ++c) grad[c * nq + k] = G[c];
      }
    }
  }
}

// adds minus the Hessian of the leaf's local expansion (coefficients scaled
// by h^|n|, so the second derivatives carry 1/h^2)
template <typename T, int P>
__global__ __launch_bounds__(FMM_BLOCK) void k_l2p_grad(DevTree t, int n,
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
  const int64_t k = t.slot[j] - off;
  const double s2 = ih * ih;
#pragma unroll
  for (int c = 0; c < 6; ++c) grad[c * nq + k] -= (double)H[c] * s2;
}

template <typename T, int KERNEL>
bool dispatch_grad(const DevTree &t, int n_nodes, int n, int p, double eps, double *grad,
                   hipStream_t s) {
  const int nb = (n + FMM_BLOCK - 1) / FMM_BLOCK;
  hipLaunchKernelGGL(k_p2p_grad<KERNEL>, dim3((n_nodes + 3) / 4), dim3(FMM_BLOCK), 0, s, t,
                     n_nodes, eps, grad, (int64_t)n, 0);
  switch (p) {
    case 1: return true;  // the Hessian of a degree-1 local expansion is zero
    case 2: hipLaunchKernelGGL((k_l2p_grad<T, 2>), dim3(nb), dim3(FMM_BLOCK), 0, s, t, n, grad, (int64_t)n, 0); return true;
    case 3: hipLaunchKernelGGL((k_l2p_grad<T, 3>), dim3(nb), dim3(FMM_BLOCK), 0, s, t, n, grad, (int64_t)n, 0); return true;
    case 4: hipLaunchKernelGGL((k_l2p_grad<T, 4>), dim3(nb), dim3(FMM_BLOCK), 0, s, t, n, grad, (int64_t)n, 0); return true;
    case 5: hipLaunchKernelGGL((k_l2p_grad<T, 5>), dim3(nb), dim3(FMM_BLOCK), 0, s, t, n, grad, (int64_t)n, 0); return true;
    case 6: hipLaunchKernelGGL((k_l2p_grad<T, 6>), dim3(nb), dim3(FMM_BLOCK), 0, s, t, n, grad, (int64_t)n, 0); return true;
    default: return false;
  }
}

}  // namespace

// One system's tree (request 0 at slot offset 0), n active particles.
hipError_t launch_force_gradient(const DevTree &t, int n_nodes, int n, int p, int kernel,
                                 bool mixed, double eps, double *grad, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  bool ok;
  if (mixed)
    ok = kernel == 1 ? dispatch_grad<float, 1>(t, n_nodes, n, p, eps, grad, s)
                     : dispatch_grad<float, 0>(t, n_nodes, n, p, eps, grad, s);
  else
    ok = kernel == 1 ? dispatch_grad<double, 1>(t, n_nodes, n, p, eps, grad, s)
                     : dispatch_grad<double, 0>(t, n_nodes, n, p, eps, grad, s);
  if (!ok) return hipErrorInvalidValue;
  return hipGetLastError();
}
