// Comoving drift and kick factors (Sec. 3.5, Eqs. 10-11): the drift operator
// advances comoving positions by (p/m) times the integral of dt/a^2 and the
// kick operator advances the canonical momenta by the force times the
// integral of dt/a, both over the step.  With x = ln a, dt = dx / H(a) and
// H(a) = H0 sqrt(Om a^-3 + Ok a^-2 + OL), Ok = 1 - Om - OL (no radiation,
// vacuum boundary).  The table holds the integrals of e^{-2x}/H and e^{-x}/H
// over each interval of a uniform grid in x; a factor between two scale
// factors is the sum of the whole intervals between them plus the two partial
// intervals at the ends, integrated with the same 8-point Gauss-Legendre rule
// (a sum of positive terms: no cancellation, unlike a difference of running
// integrals, which loses digits for short steps far from the table's start).
// Host code only: the factors are scalars of the integrator's schedule.
#include <math.h>

#include <new>
#include <vector>

#include "../../include/fmm355.h"

struct fmm_cosmo {
  fmm_cosmo_params prm;
  double x0, dx;
  std::vector<double> sd, sk;  // integrals over grid interval i (n - 1 of them)
};

namespace {

// Gauss-Legendre nodes and weights on [-1, 1], 8 points (the positive half)
const double GL_X[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267,
                        0.9602898564975363};
const double GL_W[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745,
                        0.1012285362903763};

double hubble(const fmm_cosmo_params &p, double a) {
  const double ok = 1.0 - p.omega_m - p.omega_l;
  const double e2 = p.omega_m / (a * a * a) + ok / (a * a) + p.omega_l;
  return e2 > 0 ? p.h0 * sqrt(e2) : -1.0;
}

// integrals of e^{-2x}/H (drift) and e^{-x}/H (kick) over [x1, x2]
bool segment(const fmm_cosmo_params &p, double x1, double x2, double *d, double *k) {
  const double c = 0.5 * (x1 + x2), h = 0.5 * (x2 - x1);
  double sd = 0.0, sk = 0.0;
  for (int i = 0; i < 4; ++i)
    for (int s = -1; s <= 1; s += 2) {
      const double x = c + s * h * GL_X[i];
      const double a = exp(x), H = hubble(p, a);
      if (!(H > 0)) return false;
      sd += GL_W[i] / (a * a * H);
      sk += GL_W[i] / (a * H);
    }
  *d = sd * h;
  *k = sk * h;
  return true;
}

// grid interval holding x (the last one for the upper end)
int interval(const fmm_cosmo *c, double x) {
  int i = (int)floor((x - c->x0) / c->dx);
  if (i < 0) i = 0;
  if (i > c->prm.n - 2) i = c->prm.n - 2;
  return i;
}

// factors from x0 to x1, x0 <= x1
bool forward(const fmm_cosmo *c, double x0, double x1, double *d, double *k) {
  const int i0 = interval(c, x0), i1 = interval(c, x1);
  if (i0 == i1) return segment(c->prm, x0, x1, d, k);
  double d0, k0, d1, k1;
  if (!segment(c->prm, x0, c->x0 + (i0 + 1) * c->dx, &d0, &k0) ||
      !segment(c->prm, c->x0 + i1 * c->dx, x1, &d1, &k1))
    return false;
  double sd = d0, sk = k0;
  for (int i = i0 + 1; i < i1; ++i) {
    sd += c->sd[i];
    sk += c->sk[i];
  }
  *d = sd + d1;
  *k = sk + k1;
  return true;
}

}  // namespace

extern "C" fmm_status fmm_cosmo_create(const fmm_cosmo_params *p, fmm_cosmo **out) {
  if (!p || !out) return FMM_EINVAL;
  if (!(p->h0 > 0) || !(p->a_min > 0) || !(p->a_max > p->a_min) || p->n < 2 ||
      p->n > (1 << 24) || !(p->omega_m >= 0) || !std::isfinite(p->omega_l))
    return FMM_EINVAL;
  fmm_cosmo *c = new (std::nothrow) fmm_cosmo();
  if (!c) return FMM_ENOMEM;
  c->prm = *p;
  c->x0 = log(p->a_min);
  c->dx = (log(p->a_max) - c->x0) / (p->n - 1);
  c->sd.assign(p->n - 1, 0.0);
  c->sk.assign(p->n - 1, 0.0);
  for (int i = 0; i < p->n - 1; ++i)
    if (!segment(*p, c->x0 + i * c->dx, c->x0 + (i + 1) * c->dx, &c->sd[i], &c->sk[i])) {
      delete c;
      return FMM_EINVAL;  // H^2 <= 0 inside the range
    }
  *out = c;
  return FMM_OK;
}

extern "C" fmm_status fmm_cosmo_factors(const fmm_cosmo *c, double a0, double a1, double *drift,
                                        double *kick) {
  if (!c || !drift || !kick) return FMM_EINVAL;
  const double lo = c->prm.a_min, hi = c->prm.a_max;
  if (!(a0 >= lo && a0 <= hi && a1 >= lo && a1 <= hi)) return FMM_EINVAL;
  const double x0 = log(a0), x1 = log(a1);
  double d, k;
  if (!(x0 <= x1 ? forward(c, x0, x1, &d, &k) : forward(c, x1, x0, &d, &k))) return FMM_EINVAL;
  *drift = x0 <= x1 ? d : -d;
  *kick = x0 <= x1 ? k : -k;
  return FMM_OK;
}

double cosmo_hubble(const fmm_cosmo *c, double a) { return hubble(c->prm, a); }

extern "C" fmm_status fmm_cosmo_destroy(fmm_cosmo *c) {
  if (!c) return FMM_EINVAL;
  delete c;
  return FMM_OK;
}
