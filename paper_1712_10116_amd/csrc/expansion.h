// Cartesian Taylor expansions of total degree <= P, unrolled at compile time.
//
// Multi-indices k = (kx, ky, kz), |k| <= P, are enumerated by degree, then by
// kz, then by ky (K = C(P+3,3) terms).  Every loop over them is fully unrolled
// so coefficient arrays live in registers.
//
// All coefficients are stored scaled by the cell half side h:
//   multipole  Mt[k] = sum_j m_j (u_j/h)^k / k!              (u_j = x_j - z)
//   local      Lt[n] = h^|n| d^n Phi / dx^n (z) / ...        (so that
//              Phi(z+u) = sum_n Lt[n] (u/h)^n / n!)
// which keeps FP32 values O(mass) at any tree depth.
//
// Derivatives D^k psi(R) of psi(R) = -(|R|^2 + e2)^(-1/2) come from the
// recursion for derivatives of a function of |R|^2 (McMurchie-Davidson form):
//   G_0 = -s^(-1/2),  G_{n+1} = -(2n+1) G_n / s,   s = |R|^2 + e2
//   R^n_000 = G_n,  R^n_{k+e_x} = X R^{n+1}_k + k_x R^{n+1}_{k-e_x}  (same for y, z)
//   D^k psi = R^0_k.
#pragma once
#include <hip/hip_runtime.h>

template <int P>
struct MI {
  static constexpr int K = (P + 1) * (P + 2) * (P + 3) / 6;
  int x[K], y[K], z[K], deg[K];
  int idx[P + 1][P + 1][P + 1];
  constexpr MI() : x(), y(), z(), deg(), idx() {
    for (int a = 0; a <= P; ++a)
      for (int b = 0; b <= P; ++b)
        for (int c = 0; c <= P; ++c) idx[a][b][c] = -1;
    int t = 0;
    for (int d = 0; d <= P; ++d)
      for (int c = 0; c <= d; ++c)
        for (int b = 0; b <= d - c; ++b) {
          int a = d - c - b;
          x[t] = a;
          y[t] = b;
          z[t] = c;
          deg[t] = d;
          idx[a][b][c] = t;
          ++t;
        }
  }
  constexpr int at(int a, int b, int c) const {
    return (a < 0 || b < 0 || c < 0 || a + b + c > P) ? -1 : idx[a][b][c];
  }
};

// 1/n! for small n as compile-time constants
__host__ __device__ constexpr double inv_fact(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return 1.0 / f;
}

// powers u^a / a! for a = 0..P
template <typename T, int P>
__device__ __forceinline__ void pow_fact(T u, T (&pw)[P + 1]) {
  pw[0] = T(1);
#pragma unroll
  for (int a = 1; a <= P; ++a) pw[a] = pw[a - 1] * u * T(1.0 / a);
}

// mono[t] = ux^kx/kx! * uy^ky/ky! * uz^kz/kz!
template <typename T, int P>
__device__ __forceinline__ void monomials(T ux, T uy, T uz, T (&mono)[MI<P>::K]) {
  constexpr MI<P> mi{};
  T px[P + 1], py[P + 1], pz[P + 1];
  pow_fact<T, P>(ux, px);
  pow_fact<T, P>(uy, py);
  pow_fact<T, P>(uz, pz);
#pragma unroll
  for (int t = 0; t < MI<P>::K; ++t) mono[t] = px[mi.x[t]] * py[mi.y[t]] * pz[mi.z[t]];
}

template <typename T>
__device__ __forceinline__ T fast_rsqrt(T s);
template <>
__device__ __forceinline__ float fast_rsqrt<float>(float s) {
  return __builtin_amdgcn_rsqf(s);
}
template <>
__device__ __forceinline__ double fast_rsqrt<double>(double s) {
  // hardware estimate refined by two Newton steps to full double accuracy
  double y = __builtin_amdgcn_rsq(s);
  double hs = 0.5 * s;
  y = y * fma(-hs * y, y, 1.5);
  y = y * fma(-hs * y, y, 1.5);
  return y;
}

// D[t] = d^{k_t} psi / dR^{k_t}, psi = -(|R|^2 + e2)^(-1/2), for the k_t with
// z-degree <= ZMAX (the recursion for such k only uses such k; other entries
// of D are left unset)
template <typename T, int P, int ZMAX = P>
__device__ __forceinline__ void derivatives(T X, T Y, T Z, T e2, T (&D)[MI<P>::K]) {
  constexpr MI<P> mi{};
  constexpr int K = MI<P>::K;
  const T s = X * X + Y * Y + Z * Z + e2;
  const T rinv = fast_rsqrt<T>(s);
  const T sinv = rinv * rinv;
  T G[P + 1];
  G[0] = -rinv;
#pragma unroll
  for (int n = 0; n < P; ++n) G[n + 1] = T(-(2 * n + 1)) * G[n] * sinv;
  // level n holds R^n_k for |k| <= P - n; level P-1 down to 0
  T Rn[P + 1][K];
#pragma unroll
  for (int n = P; n >= 0; --n) {
#pragma unroll
    for (int t = 0; t < K; ++t) {
      const int d = mi.deg[t];
      if (d > P - n || mi.z[t] > ZMAX) continue;
      if (d == 0) {
        Rn[n][t] = G[n];
        continue;
      }
      const int a = mi.x[t], b = mi.y[t], c = mi.z[t];
      if (a > 0) {
        T v = X * Rn[n + 1][mi.at(a - 1, b, c)];
        if (a > 1) v += T(a - 1) * Rn[n + 1][mi.at(a - 2, b, c)];
        Rn[n][t] = v;
      } else if (b > 0) {
        T v = Y * Rn[n + 1][mi.at(a, b - 1, c)];
        if (b > 1) v += T(b - 1) * Rn[n + 1][mi.at(a, b - 2, c)];
        Rn[n][t] = v;
      } else {
        T v = Z * Rn[n + 1][mi.at(a, b, c - 1)];
        if (c > 1) v += T(c - 1) * Rn[n + 1][mi.at(a, b, c - 2)];
        Rn[n][t] = v;
      }
    }
  }
#pragma unroll
  for (int t = 0; t < K; ++t)
    if (mi.z[t] <= ZMAX) D[t] = Rn[0][t];
}

// Compile-time term lists: only the (n, m) index pairs that occur, so every
// unrolled step addresses registers with constant indices.
template <int P>
struct M2LTerms {  // pairs with |n| + |m| <= P:  (n, m, n+m)
  static constexpr int count() {
    constexpr MI<P> mi{};
    int c = 0;
    for (int n = 0; n < MI<P>::K; ++n)
      for (int m = 0; m < MI<P>::K; ++m) c += mi.deg[n] + mi.deg[m] <= P;
    return c;
  }
  static constexpr int NT = count();
  int n[NT], m[NT], nm[NT];
  constexpr M2LTerms() : n(), m(), nm() {
    constexpr MI<P> mi{};
    int c = 0;
    for (int a = 0; a < MI<P>::K; ++a)
      for (int b = 0; b < MI<P>::K; ++b)
        if (mi.deg[a] + mi.deg[b] <= P) {
          n[c] = a;
          m[c] = b;
          nm[c] = mi.at(mi.x[a] + mi.x[b], mi.y[a] + mi.y[b], mi.z[a] + mi.z[b]);
          ++c;
        }
  }
};

template <int P>
struct ShiftTerms {  // pairs k <= m componentwise:  (m, k, m-k)
  static constexpr int count() {
    constexpr MI<P> mi{};
    int c = 0;
    for (int m = 0; m < MI<P>::K; ++m)
      for (int k = 0; k < MI<P>::K; ++k)
        c += mi.x[k] <= mi.x[m] && mi.y[k] <= mi.y[m] && mi.z[k] <= mi.z[m];
    return c;
  }
  static constexpr int NT = count();
  int hi[NT], lo[NT], diff[NT];
  constexpr ShiftTerms() : hi(), lo(), diff() {
    constexpr MI<P> mi{};
    int c = 0;
    for (int m = 0; m < MI<P>::K; ++m)
      for (int k = 0; k < MI<P>::K; ++k)
        if (mi.x[k] <= mi.x[m] && mi.y[k] <= mi.y[m] && mi.z[k] <= mi.z[m]) {
          hi[c] = m;
          lo[c] = k;
          diff[c] = mi.at(mi.x[m] - mi.x[k], mi.y[m] - mi.y[k], mi.z[m] - mi.z[k]);
          ++c;
        }
  }
};

// Lacc[n] += sum_{|n|+|m|<=P} Ms[m] D[n+m]
template <typename T, int P>
__device__ __forceinline__ void m2l_contract(const T (&Ms)[MI<P>::K], const T (&D)[MI<P>::K],
                                             T (&Lacc)[MI<P>::K]) {
  constexpr M2LTerms<P> tt{};
#pragma unroll
  for (int q = 0; q < M2LTerms<P>::NT; ++q) Lacc[tt.n[q]] = fma(Ms[tt.m[q]], D[tt.nm[q]], Lacc[tt.n[q]]);
}

// ---------------------------------------------------------------------------
// Harmonic far field.  For psi = -1/|R| the derivative tensors satisfy
// Laplace's equation, D[k + 2e_z] = -D[k + 2e_x] - D[k + 2e_y], so in
//   L[n] = sum_m M[m] D[n+m]
// every moment with m_z >= 2 can be moved onto two moments of the same degree
// with m_z lowered by 2 ("folding"), leaving the 2d+1 moments of each degree d
// with m_z <= 1.  The local coefficients obey the same relation, so only the
// 2d+1 with n_z <= 1 need the contraction; the rest follow by "unfolding".
// Per pair this costs sum_{a+b<=P} (2a+1)(2b+1) multiply-adds instead of
// C(P+6,6) (532 instead of 924 at P = 6), with derivatives of z-degree <= 2.
// ---------------------------------------------------------------------------
template <int P>
struct HI {  // the multi-indices with z-degree <= 1, in MI order
  static constexpr int KH = (P + 1) * (P + 1);
  int full[KH];            // compact -> MI index
  int compact[MI<P>::K];   // MI index -> compact index, or -1
  constexpr HI() : full(), compact() {
    constexpr MI<P> mi{};
    int c = 0;
    for (int t = 0; t < MI<P>::K; ++t) {
      compact[t] = mi.z[t] <= 1 ? c : -1;
      if (mi.z[t] <= 1) full[c++] = t;
    }
  }
};

// moments folded onto z-degree <= 1: Mh[compact(m)] for m_z <= 1
template <typename T, int P>
__device__ __forceinline__ void fold_moments(const T (&M)[MI<P>::K], T (&Mh)[HI<P>::KH]) {
  constexpr MI<P> mi{};
  constexpr HI<P> hi{};
  T w[MI<P>::K];
#pragma unroll
  for (int t = 0; t < MI<P>::K; ++t) w[t] = M[t];
  // within each degree, highest z first, so folded values cascade down by 2
#pragma unroll
  for (int d = 2; d <= P; ++d)
#pragma unroll
    for (int c = d; c >= 2; --c)
#pragma unroll
      for (int b = 0; b <= d - c; ++b) {
        const int a = d - c - b;
        const int t = mi.at(a, b, c);
        w[mi.at(a + 2, b, c - 2)] -= w[t];
        w[mi.at(a, b + 2, c - 2)] -= w[t];
      }
#pragma unroll
  for (int j = 0; j < HI<P>::KH; ++j) Mh[j] = w[hi.full[j]];
}

// local coefficients with n_z >= 2 from those with lower n_z (same degree)
template <typename T, int P>
__device__ __forceinline__ void unfold_locals(T (&L)[MI<P>::K]) {
  constexpr MI<P> mi{};
#pragma unroll
  for (int d = 2; d <= P; ++d)
#pragma unroll
    for (int c = 2; c <= d; ++c)
#pragma unroll
      for (int b = 0; b <= d - c; ++b) {
        const int a = d - c - b;
        L[mi.at(a, b, c)] = -L[mi.at(a + 2, b, c - 2)] - L[mi.at(a, b + 2, c - 2)];
      }
}

template <int P>
struct M2LHTerms {  // (n, m) with n_z, m_z <= 1 and |n| + |m| <= P: (n, compact m, n+m)
  static constexpr int count() {
    constexpr MI<P> mi{};
    int c = 0;
    for (int n = 0; n < MI<P>::K; ++n)
      for (int m = 0; m < MI<P>::K; ++m)
        c += mi.z[n] <= 1 && mi.z[m] <= 1 && mi.deg[n] + mi.deg[m] <= P;
    return c;
  }
  static constexpr int NT = count();
  int n[NT], mc[NT], nm[NT];
  constexpr M2LHTerms() : n(), mc(), nm() {
    constexpr MI<P> mi{};
    constexpr HI<P> hi{};
    int c = 0;
    for (int a = 0; a < MI<P>::K; ++a)
      for (int b = 0; b < MI<P>::K; ++b)
        if (mi.z[a] <= 1 && mi.z[b] <= 1 && mi.deg[a] + mi.deg[b] <= P) {
          n[c] = a;
          mc[c] = hi.compact[b];
          nm[c] = mi.at(mi.x[a] + mi.x[b], mi.y[a] + mi.y[b], mi.z[a] + mi.z[b]);
          ++c;
        }
  }
};

// Lacc[n] += sum_m Mh[m] D[n+m] over n_z, m_z <= 1 (Lacc entries with n_z >= 2 untouched)
template <typename T, int P>
__device__ __forceinline__ void m2l_contract_h(const T (&Mh)[HI<P>::KH], const T (&D)[MI<P>::K],
                                               T (&Lacc)[MI<P>::K]) {
  constexpr M2LHTerms<P> tt{};
#pragma unroll
  for (int q = 0; q < M2LHTerms<P>::NT; ++q)
    Lacc[tt.n[q]] = fma(Mh[tt.mc[q]], D[tt.nm[q]], Lacc[tt.n[q]]);
}

// Multipole shift to the parent: Mp[m] += sum_{k<=m} beta^|k| Mc[k] q[m-k],
// q = monomials((z_c - z_p)/h_p), beta = h_c/h_p.
template <typename T, int P>
__device__ __forceinline__ void m2m_shift(const T (&Mc)[MI<P>::K], T beta, const T (&q)[MI<P>::K],
                                          T (&Mp)[MI<P>::K]) {
  constexpr MI<P> mi{};
  constexpr ShiftTerms<P> tt{};
  constexpr int K = MI<P>::K;
  T bp[P + 1];
  bp[0] = T(1);
#pragma unroll
  for (int d = 1; d <= P; ++d) bp[d] = bp[d - 1] * beta;
  T Mb[K];
#pragma unroll
  for (int k = 0; k < K; ++k) Mb[k] = Mc[k] * bp[mi.deg[k]];
#pragma unroll
  for (int t = 0; t < ShiftTerms<P>::NT; ++t) Mp[tt.hi[t]] = fma(Mb[tt.lo[t]], q[tt.diff[t]], Mp[tt.hi[t]]);
}

// Local shift to a child: Lc[n] += gamma^|n| sum_{k>=n} Lp[k] q[k-n],
// q = monomials((z_c - z_p)/h_p), gamma = h_c/h_p.
template <typename T, int P>
__device__ __forceinline__ void l2l_shift(const T (&Lp)[MI<P>::K], T gamma, const T (&q)[MI<P>::K],
                                          T (&Lc)[MI<P>::K]) {
  constexpr MI<P> mi{};
  constexpr ShiftTerms<P> tt{};
  constexpr int K = MI<P>::K;
  T gp[P + 1];
  gp[0] = T(1);
#pragma unroll
  for (int d = 1; d <= P; ++d) gp[d] = gp[d - 1] * gamma;
  T acc[K];
#pragma unroll
  for (int n = 0; n < K; ++n) acc[n] = T(0);
  // term (hi=k, lo=n, diff=k-n): acc[n] += Lp[k] q[k-n]
#pragma unroll
  for (int t = 0; t < ShiftTerms<P>::NT; ++t) acc[tt.lo[t]] = fma(Lp[tt.hi[t]], q[tt.diff[t]], acc[tt.lo[t]]);
#pragma unroll
  for (int n = 0; n < K; ++n) Lc[n] = fma(gp[mi.deg[n]], acc[n], Lc[n]);
}

// Potential and minus gradient (per unit h) of a local expansion at u/h:
// phi = sum_n Lt[n] mono[n];  g_d = sum_{|n|<P} Lt[n+e_d] mono[n]
template <typename T, int P>
__device__ __forceinline__ void l2p_eval(const T (&Lt)[MI<P>::K], const T (&mono)[MI<P>::K],
                                         T &phi, T &gx, T &gy, T &gz) {
  constexpr MI<P> mi{};
  constexpr int K = MI<P>::K;
  phi = gx = gy = gz = T(0);
#pragma unroll
  for (int n = 0; n < K; ++n) {
    phi = fma(Lt[n], mono[n], phi);
    if (mi.deg[n] < P) {
      gx = fma(Lt[mi.at(mi.x[n] + 1, mi.y[n], mi.z[n])], mono[n], gx);
      gy = fma(Lt[mi.at(mi.x[n], mi.y[n] + 1, mi.z[n])], mono[n], gy);
      gz = fma(Lt[mi.at(mi.x[n], mi.y[n], mi.z[n] + 1)], mono[n], gz);
    }
  }
}
