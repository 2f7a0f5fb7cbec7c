// Forward fourth-order integrator of Chin & Chen (2005), the higher-order
// alternative to the KDK leapfrog that Sec. 4.1 proposes, with one shared
// timestep h.  Their algorithm 4A, a factorisation of exp(h (T + V)) with
// positive steps only, kicks with h/6, drifts h/2, kicks with 2h/3 under a
// modified potential, drifts h/2 and kicks h/6.  The modified kick uses
//     a~_i = a_i + (h^2 / 24) sum_j (d a_i / d x_j) a_j
//          = a_i + (h^2 / 24) (T_i a_i + u_i),
// T_i = d a_i / d x_i the force gradient (fmm_forces_grad) and
// u_i = sum_{j != i} m_j H(x_i - x_j) a_j the field of the vector sources
// m_j a_j (fmm_evaluate_dipole on the same tree): the derivative of a_i along
// a displacement of every particle by its own acceleration.  Kicks and drifts
// are FP64; both force evaluations of a step are complete FMM solves, so the
// pair symmetry of the solver makes sum_i m_i (T_i a_i + u_i) vanish and the
// scheme conserves momentum like the KDK.
#include "../../include/fmm355.h"
#include "common.h"
#include "context.h"

namespace {

// y[k] += c x[k] for k < m
__global__ __launch_bounds__(FMM_BLOCK) void k_axpy(double *__restrict__ y,
                                                    const double *__restrict__ x, int64_t m,
                                                    double c) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) y[k] = y[k] + c * x[k];
}

// v += c3 (a + c2 (T a + u)), T symmetric from its rows xx, yy, zz, xy, xz, yz
__global__ __launch_bounds__(FMM_BLOCK) void k_chin_kick(double *__restrict__ vel,
                                                         const double *__restrict__ a,
                                                         const double *__restrict__ T,
                                                         const double *__restrict__ u,
                                                         int64_t n, double c2, double c3) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double ax = a[i], ay = a[n + i], az = a[2 * n + i];
  const double txx = T[i], tyy = T[n + i], tzz = T[2 * n + i];
  const double txy = T[3 * n + i], txz = T[4 * n + i], tyz = T[5 * n + i];
  const double gx = (txx * ax + txy * ay) + txz * az;
  const double gy = (txy * ax + tyy * ay) + tyz * az;
  const double gz = (txz * ax + tyz * ay) + tzz * az;
  vel[i] = vel[i] + c3 * (ax + c2 * (gx + u[i]));
  vel[n + i] = vel[n + i] + c3 * (ay + c2 * (gy + u[n + i]));
  vel[2 * n + i] = vel[2 * n + i] + c3 * (az + c2 * (gz + u[2 * n + i]));
}

void axpy(double *y, const double *x, int64_t m, double c, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, dim3((unsigned)((m + FMM_BLOCK - 1) / FMM_BLOCK)), dim3(FMM_BLOCK),
                     0, s, y, x, m, c);
}

fmm_status check_state(fmm_ctx *c, const chin_state *st) {
  if (!c || !st) return FMM_EINVAL;
  if (st->n < 1 || st->n > c->max_n || !st->pos || !st->vel || !st->mass || !st->acc ||
      !st->work)
    return fmm_fail(c, FMM_EINVAL, "chin: bad state (n=%lld, max_n=%lld, NULL array)",
                    (long long)st->n, (long long)c->max_n);
  return FMM_OK;
}

}  // namespace

extern "C" int64_t chin_work_bytes(int64_t n) {
  return n < 1 ? -1 : 13 * n * (int64_t)sizeof(double);
}

extern "C" fmm_status chin_init(fmm_ctx *c, chin_state *st, double eps, double theta, int p) {
  fmm_status s = check_state(c, st);
  if (s != FMM_OK) return s;
  const int64_t n = st->n;
  return fmm_forces(c, st->pos, st->mass, n, nullptr, n, eps, theta, p, st->acc,
                    st->work + 12 * n);
}

extern "C" fmm_status chin_step(fmm_ctx *c, chin_state *st, double eps, double theta, int p,
                                double h, int64_t stats[3]) {
  fmm_status s = check_state(c, st);
  if (s != FMM_OK) return s;
  if (!(h == h) || h == 0.0 || h - h != 0.0) return fmm_fail(c, FMM_EINVAL, "chin: bad step");
  const int64_t n = st->n;
  double *amid = st->work, *grad = st->work + 3 * n, *u = st->work + 9 * n,
         *pot = st->work + 12 * n;
  hipStream_t hs = c->stream;
  axpy(st->vel, st->acc, 3 * n, h / 6, hs);  // opening kick, h/6
  axpy(st->pos, st->vel, 3 * n, h / 2, hs);  // drift, h/2
  s = fmm_forces_grad(c, st->pos, st->mass, n, nullptr, n, eps, theta, p, amid, pot, grad);
  if (s != FMM_OK) return s;
  s = fmm_evaluate_dipole(c, st->pos, st->mass, n, nullptr, n, p, amid, u, pot);
  if (s != FMM_OK) return s;
  hipLaunchKernelGGL(k_chin_kick, dim3((unsigned)((n + FMM_BLOCK - 1) / FMM_BLOCK)),
                     dim3(FMM_BLOCK), 0, hs, st->vel, amid, grad, u, n, (h * h) / 24,
                     (2 * h) / 3);  // modified kick, 2h/3
  axpy(st->pos, st->vel, 3 * n, h / 2, hs);  // drift, h/2
  s = fmm_forces(c, st->pos, st->mass, n, nullptr, n, eps, theta, p, st->acc, pot);
  if (s != FMM_OK) return s;
  axpy(st->vel, st->acc, 3 * n, h / 6, hs);  // closing kick, h/6
  if (hipGetLastError() != hipSuccess) return fmm_fail(c, FMM_EDEVICE, "chin: launch failed");
  st->t += h;
  if (stats) {
    stats[0] = 3;
    stats[1] = 3 * n;
    stats[2] = 2;
  }
  return FMM_OK;
}
