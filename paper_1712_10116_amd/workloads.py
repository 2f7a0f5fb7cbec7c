"""Seeded synthetic particle sets with the shapes of the paper's workloads.

This module only draws inputs; it holds none of the force-solve arithmetic.
Both the GPU path and the CPU oracle are fed from here.  Every generator is
deterministic for a given seed (numpy ``default_rng``).  Positions and
velocities are float64 SoA arrays of shape (3, n); masses float64 (n,).
G = 1 throughout.

Stand-ins: the paper's own initial conditions (the isolated disk galaxy of
Sec. 3.4 and the Aquarius zoom of Sec. 3.5) are not available, so the disk and
zoom generators below draw particle sets of the same kind and size class.
"""
from __future__ import annotations

import functools

import numpy as np

_N_CONFIG = {0: 4096, 1: 1 << 20, 2: 1 << 22, 3: 1 << 24}


def _isotropic(rng, n):
    cz = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    sz = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    return np.stack([sz * np.cos(ph), sz * np.sin(ph), cz])


def _recentre(pos, vel, mass):
    mtot = mass.sum()
    pos = pos - (pos * mass).sum(axis=1, keepdims=True) / mtot
    vel = vel - (vel * mass).sum(axis=1, keepdims=True) / mtot
    return pos, vel


def plummer(n, seed=1000, a=1.0, mtot=1.0, rmax_frac=0.999):
    """Plummer sphere, G = M = a = 1 by default, isotropic velocities drawn from
    the Plummer distribution function (rejection sampling of q^2 (1-q^2)^(7/2))."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.0, rmax_frac, n)
    X = np.where(X <= 0.0, 1e-12, X)
    r = a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    pos = r * _isotropic(rng, n)
    q = np.empty(n)
    filled = 0
    while filled < n:
        m = 2 * (n - filled) + 16
        qq = rng.uniform(0.0, 1.0, m)
        yy = rng.uniform(0.0, 0.1, m)
        ok = qq[yy < qq * qq * (1.0 - qq * qq) ** 3.5]
        take = min(len(ok), n - filled)
        q[filled:filled + take] = ok[:take]
        filled += take
    vesc = np.sqrt(2.0 * mtot / a) * (1.0 + (r / a) ** 2) ** (-0.25)
    vel = (q * vesc) * _isotropic(rng, n)
    mass = np.full(n, mtot / n)
    pos, vel = _recentre(pos, vel, mass)
    return pos, vel, mass


def uniform_sphere(n, seed=1001, radius=1.0, mtot=1.0):
    """Cold collapse initial condition: uniform in a sphere, at rest."""
    rng = np.random.default_rng(seed)
    r = radius * rng.uniform(0.0, 1.0, n) ** (1.0 / 3.0)
    pos = r * _isotropic(rng, n)
    vel = np.zeros((3, n))
    mass = np.full(n, mtot / n)
    return pos, vel, mass


def _inv_cdf(cdf, x_hi, u, n_grid=20000):
    xs = np.linspace(0.0, x_hi, n_grid)
    cs = cdf(xs)
    cs = cs / cs[-1]
    return np.interp(u, cs, xs)


def _nfw_radii(rng, n, rs, c):
    m = lambda x: np.log1p(x) - x / (1.0 + x)
    return rs * _inv_cdf(m, c, rng.uniform(0.0, 1.0, n))


def disk_galaxy(n=1 << 22, seed=1002):
    """Exponential disk (1/4 of n, scale length 1, sech^2 height 0.1, R <= 10),
    Hernquist bulge (1/8, a = 0.2), NFW halo (5/8, c = 10, r_s = 6, cut at
    20 r_s); halo particles 8x heavier than disk/bulge ones; total mass 1."""
    rng = np.random.default_rng(seed)
    nd, nb = n // 4, n // 8
    nh = n - nd - nb
    R = _inv_cdf(lambda x: 1.0 - (1.0 + x) * np.exp(-x), 10.0, rng.uniform(0, 1, nd))
    ph = rng.uniform(0.0, 2.0 * np.pi, nd)
    zd = 0.1 * np.arctanh(np.clip(2.0 * rng.uniform(0, 1, nd) - 1.0, -0.999999, 0.999999))
    pd = np.stack([R * np.cos(ph), R * np.sin(ph), zd])
    sb = np.sqrt(rng.uniform(0, 1, nb) * 0.999)
    rb = 0.2 * sb / (1.0 - sb)
    pb = rb * _isotropic(rng, nb)
    rh = _nfw_radii(rng, nh, 6.0, 20.0)
    phh = rh * _isotropic(rng, nh)
    pos = np.concatenate([pd, pb, phh], axis=1)
    w = np.concatenate([np.ones(nd + nb), np.full(nh, 8.0)])
    mass = w / w.sum()
    rr = np.sqrt((pos * pos).sum(axis=0))
    order = np.argsort(rr)
    menc = np.empty(n)
    menc[order] = np.cumsum(mass[order])
    vc = np.sqrt(menc / np.maximum(rr, 1e-3))
    vel = 0.1 * vc * rng.standard_normal((3, n))
    tang = np.stack([-pd[1], pd[0], np.zeros(nd)]) / np.maximum(R, 1e-6)
    vel[:, :nd] += vc[:nd] * tang
    pos, vel = _recentre(pos, vel, mass)
    return pos, vel, mass


def clustered_zoom(n=1 << 24, seed=1003, n_halos=2000):
    """2000 NFW halos (c = 10) with masses from dN/dM ~ M^-1.9 on [1, 1e3],
    particle counts proportional to halo mass over 80% of n, centred uniformly
    in [0.25, 0.75]^3, r_200 = 0.05 (M/M_max)^(1/3); plus a uniform background
    of 20% of n in [0, 1]^3 with 8x heavier particles."""
    rng = np.random.default_rng(seed)
    n_bg = n // 5
    n_h = n - n_bg
    u = rng.uniform(0, 1, n_halos)
    a = -0.9
    Mh = (1.0 + u * (1e3 ** a - 1.0)) ** (1.0 / a)
    counts = np.floor(Mh / Mh.sum() * n_h).astype(np.int64)
    counts[np.argmax(Mh)] += n_h - counts.sum()
    centres = rng.uniform(0.25, 0.75, (3, n_halos))
    r200 = 0.05 * (Mh / Mh.max()) ** (1.0 / 3.0)
    parts = []
    for h in range(n_halos):
        k = int(counts[h])
        if k == 0:
            continue
        r = _nfw_radii(rng, k, r200[h] / 10.0, 10.0)
        parts.append(centres[:, h:h + 1] + r * _isotropic(rng, k))
    pos = np.concatenate(parts + [rng.uniform(0.0, 1.0, (3, n_bg))], axis=1)
    mass = np.concatenate([np.ones(n_h), np.full(n_bg, 8.0)])
    mass = mass / mass.sum()
    vel = 0.1 * rng.standard_normal((3, n))
    return pos, vel, mass


@functools.lru_cache(maxsize=8)
def _king_profile(w0):
    """Tabulated King model: radius, dimensionless potential W and cumulative
    mass (in units of 9 int r^2 rho/rho0 dr) from the Poisson equation
    W'' + (2/r) W' = -9 rho(W)/rho0 (fourth-order Runge-Kutta)."""
    from math import erf

    def rho_of_w(w):
        if w <= 0:
            return 0.0
        return np.exp(w) * erf(np.sqrt(w)) - np.sqrt(4.0 * w / np.pi) * (1.0 + 2.0 * w / 3.0)

    rho0 = rho_of_w(w0)

    def f(rr, y):
        return np.array([y[1], -9.0 * rho_of_w(y[0]) / rho0 - 2.0 * y[1] / rr])

    h = 2e-3
    r, y = 1e-6, np.array([w0, 0.0])
    rs, ws, ms = [0.0], [w0], [0.0]
    m = 0.0
    while y[0] > 0 and r < 1e3:
        k1 = f(r, y); k2 = f(r + h / 2, y + h / 2 * k1)
        k3 = f(r + h / 2, y + h / 2 * k2); k4 = f(r + h, y + h * k3)
        m += r * r * rho_of_w(y[0]) / rho0 * h
        y = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        r += h
        rs.append(r); ws.append(max(float(y[0]), 0.0)); ms.append(m)
    return np.array(rs), np.array(ws), np.array(ms)


def king(n, seed=5001, w0=6.0, henon=False):
    """King (1966) model with central dimensionless potential W0, drawn from
    its distribution function f(E) ~ exp(W - v^2/2) - 1 (sigma = 1, King radius
    1), then rescaled to unit total mass with G = 1.  Radii follow the tabulated
    cumulative mass of the integrated Poisson equation
    W'' + (2/r) W' = -9 rho(W)/rho0; speeds are drawn by vectorised rejection
    sampling of v^2 (exp(W - v^2/2) - 1) on [0, sqrt(2W)].  With henon=True
    lengths and velocities are rescaled to Henon units (potential energy -1/2
    for M = G = 1), the potential energy taken from the tabulated profile."""
    rng = np.random.default_rng(seed)
    rs, ws, ms = _king_profile(float(w0))
    radii = np.interp(rng.uniform(0, 1, n) * ms[-1], ms, rs)
    W = np.interp(radii, rs, ws)
    vmax = np.sqrt(2.0 * W)
    fmax = vmax * vmax * np.expm1(W) + 1e-300
    sp = np.zeros(n)
    todo = np.arange(n)
    while len(todo):
        v = rng.uniform(0.0, 1.0, len(todo)) * vmax[todo]
        y2 = rng.uniform(0.0, 1.0, len(todo)) * fmax[todo]
        ok = y2 < v * v * np.expm1(W[todo] - 0.5 * v * v)
        sp[todo[ok]] = v[ok]
        todo = todo[~ok]
    pos = radii * _isotropic(rng, n)
    vel = sp * _isotropic(rng, n)
    mass = np.full(n, 1.0 / n)
    # with G = sigma = r0 = 1 the model mass is 9 * int r^2 rho/rho0 dr; scale
    # velocities by sqrt(M_new / M_model) to reach unit mass at fixed radii
    vel *= 1.0 / np.sqrt(9.0 * ms[-1])
    if henon:
        # W = -int G M(r) / r dM over the unit-mass profile; Henon units have
        # W = -1/2, reached by r -> r (-2 W) and v -> v / sqrt(-2 W)
        mm = ms / ms[-1]
        rm = 0.5 * (rs[1:] + rs[:-1])
        wpot = -np.sum(0.5 * (mm[1:] + mm[:-1]) / rm * np.diff(mm))
        scale = -2.0 * wpot
        pos = pos * scale
        vel = vel / np.sqrt(scale)
    pos, vel = _recentre(pos, vel, mass)
    return pos, vel, mass


def ensemble_request(i, n_min=1024, n_max=262144):
    """Request i of the serving ensemble: N log-uniform in [n_min, n_max]
    (seed 5000 + i), a Plummer sphere for even i and a King W0 = 6 model for
    odd i, both in Henon units (Plummer scale length 3 pi / 16)."""
    seed = 5000 + i
    n = int(round(np.exp(np.random.default_rng(seed).uniform(np.log(n_min), np.log(n_max)))))
    if i % 2 == 0:
        return plummer(n, seed=seed, a=3.0 * np.pi / 16.0)
    return king(n, seed=seed, henon=True)


def config(idx, n=None):
    """Particle set of one named workload: 0 Plummer 4096, 1 cold collapse 2^20,
    2 disk galaxy 2^22, 3 clustered zoom 2^24 (n may override the size)."""
    seed = 1000 + idx
    nn = n if n is not None else _N_CONFIG[idx]
    if idx == 0:
        return plummer(nn, seed=seed)
    if idx == 1:
        return uniform_sphere(nn, seed=seed)
    if idx == 2:
        return disk_galaxy(nn, seed=seed)
    if idx == 3:
        return clustered_zoom(nn, seed=seed)
    raise ValueError(idx)


# solver parameters of each workload (kernel: 0 Wendland C2, 1 Plummer).
# Timesteps are sqrt(eta*eps/|a|); eta = 0.0025 is the workload's stated
# 0.05*sqrt(eps/|a|) written in that form.
PARAMS = {
    0: dict(p=4, theta=0.5, eps=0.01, leaf_size=16, kernel=1, eta=0.0025, max_levels=10),
    1: dict(p=4, theta=0.5, eps=0.005, leaf_size=16, kernel=0, eta=0.0025, max_levels=10),
    2: dict(p=6, theta=0.4, eps=0.02, leaf_size=16, kernel=0, eta=0.0025, max_levels=14),
    3: dict(p=6, theta=0.4, eps=0.001, leaf_size=16, kernel=0, eta=0.0025, max_levels=16),
    4: dict(p=4, theta=0.5, eps=0.01, leaf_size=16, kernel=0, eta=0.0025, max_levels=10),
}
