"""Pins of the oracle's pair kernels and expansion derivatives against facts the
mathematics fixes (no GPU).  The Wendland C2 kernel is Eq. (8) of the paper;
its defining properties -- it joins -1/r at u = 1 with continuous first and
second derivatives and is the potential of a unit mass -- are checked by
finite differences and Gauss's law rather than by retyping the polynomial."""
import json
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("eps", [0.01, 0.5, 1.0, 3.0])
def test_wendland_closed_forms(oracle, eps):
    phi = lambda r: oracle.kernel_phi(oracle.WENDLAND, r, eps)
    g = lambda r: oracle.kernel_g(oracle.WENDLAND, r, eps)
    # value at the origin and at the softening length
    assert phi(0.0) == pytest.approx(-3.0 / eps, rel=1e-14)
    assert phi(eps) == pytest.approx(-1.0 / eps, rel=1e-14)
    # continuity of phi, phi' and phi'' across u = 1 (C2 join with -1/r)
    h = eps * 1e-6
    for f in (phi,):
        assert f(eps - h) == pytest.approx(f(eps + h), rel=1e-5)
    d1 = lambda r: (phi(r + h) - phi(r - h)) / (2 * h)
    assert d1(eps - 4 * h) == pytest.approx(1.0 / eps ** 2, rel=1e-4)
    # second derivative just inside and just outside u = 1 agree (C2); a join
    # that were only C1 would leave an O(1) jump here
    dl = 1e-3
    h2 = dl * eps / 10
    d2 = lambda r: (phi(r + h2) - 2 * phi(r) + phi(r - h2)) / (h2 * h2)
    assert d2(eps * (1 - dl)) == pytest.approx(d2(eps * (1 + dl)), rel=2e-2)
    assert d2(eps * (1 + dl)) == pytest.approx(-2.0 / (eps * (1 + dl)) ** 3, rel=1e-4)
    # g is phi'(r)/r everywhere, checked by central differences
    for u in (0.05, 0.3, 0.7, 0.95, 1.5, 4.0):
        r = u * eps
        hh = r * 1e-6
        fd = (phi(r + hh) - phi(r - hh)) / (2 * hh)
        assert g(r) * r == pytest.approx(fd, rel=1e-6)
    # force continuity and unit enclosed mass (Gauss): eps^2 * phi'(eps) = 1
    assert g(eps) * eps ** 3 == pytest.approx(1.0, rel=1e-13)


def test_wendland_unit_mass_density(oracle):
    # rho = lap(phi) / (4 pi) integrated over the ball must be 1; lap(phi) of a
    # radial function is phi'' + 2 phi'/r, done here by finite differences.
    eps = 0.7
    phi = lambda r: oracle.kernel_phi(oracle.WENDLAND, r, eps)
    rs = np.linspace(1e-4, eps, 4001)
    h = 1e-5
    lap = np.array([(phi(r + h) - 2 * phi(r) + phi(r - h)) / h ** 2
                    + 2.0 / r * (phi(r + h) - phi(r - h)) / (2 * h) for r in rs])
    mass = np.trapezoid(rs ** 2 * lap, rs)   # int 4 pi r^2 (lap/4pi) dr
    assert mass == pytest.approx(1.0, rel=1e-4)
    # density must be non-negative (a physical mass distribution)
    assert (lap[:-5] > -1e-4 * lap[0]).all()


def test_wendland_golden_points(oracle):
    with open(os.path.join(GOLDEN, "wendland_eq8.json")) as f:
        gold = json.load(f)
    eps = gold["eps"]
    for u, val in gold["phi_times_eps"]:
        assert oracle.kernel_phi(oracle.WENDLAND, u * eps, eps) * eps == pytest.approx(val, abs=1e-15)


@pytest.mark.parametrize("eps", [0.01, 0.3])
def test_plummer_textbook(oracle, eps):
    for r in (0.0, 0.001, 0.1, 1.0, 10.0):
        assert oracle.kernel_phi(oracle.PLUMMER, r, eps) == pytest.approx(-1.0 / math.sqrt(r * r + eps * eps), rel=1e-15)
        if r > 0:
            h = max(r, eps) * 1e-5
            fd = (oracle.kernel_phi(oracle.PLUMMER, r + h, eps) - oracle.kernel_phi(oracle.PLUMMER, r - h, eps)) / (2 * h)
            assert oracle.kernel_g(oracle.PLUMMER, r, eps) * r == pytest.approx(fd, rel=1e-6)


def _dict(D, k):
    return {tuple(int(x) for x in kk): D[i] for i, kk in enumerate(k)}


@pytest.mark.parametrize("R", [(0.3, -1.2, 0.7), (2.0, 0.1, -0.4), (-0.05, 0.02, 0.9)])
def test_derivs_closed_forms_order2(oracle, R):
    R = np.array(R)
    D, k = oracle.derivs(2, R)
    d = _dict(D, k)
    r = np.linalg.norm(R)
    assert d[(0, 0, 0)] == pytest.approx(-1.0 / r, rel=1e-14)
    for a in range(3):
        e = [0, 0, 0]; e[a] = 1
        assert d[tuple(e)] == pytest.approx(R[a] / r ** 3, rel=1e-13)
        for b in range(3):
            ee = [0, 0, 0]; ee[a] += 1; ee[b] += 1
            want = ((a == b) * r * r - 3 * R[a] * R[b]) / r ** 5
            assert d[tuple(ee)] == pytest.approx(want, rel=1e-12, abs=1e-12 / r ** 3)


@pytest.mark.parametrize("p", [4, 6, 8])
def test_derivs_harmonic_trace(oracle, p):
    # -1/r is harmonic: sum_d D^{k+2e_d} = 0 for every |k| <= p-2
    R = np.array([0.4, -0.9, 1.3])
    D, k = oracle.derivs(p, R)
    d = _dict(D, k)
    scale = max(abs(x) for x in D)
    for kk in d:
        if sum(kk) <= p - 2:
            tr = sum(d[tuple(kk[i] + 2 * (i == a) for i in range(3))] for a in range(3))
            assert abs(tr) < 1e-11 * scale


@pytest.mark.parametrize("e2", [0.0, 0.04])
def test_derivs_finite_difference(oracle, e2):
    # D^{k+e_a}(R) = d/dR_a D^k(R), checked by central differences up to degree 6
    p = 6
    R = np.array([0.8, 0.5, -0.6])
    D, k = oracle.derivs(p, R, e2)
    d = _dict(D, k)
    h = 1e-5
    for a in range(3):
        Rp = R.copy(); Rp[a] += h
        Rm = R.copy(); Rm[a] -= h
        dp_, _ = oracle.derivs(p, Rp, e2)
        dm_, _ = oracle.derivs(p, Rm, e2)
        dp_, dm_ = _dict(dp_, k), _dict(dm_, k)
        for kk in d:
            if sum(kk) < p:
                up = tuple(kk[i] + (i == a) for i in range(3))
                fd = (dp_[kk] - dm_[kk]) / (2 * h)
                assert fd == pytest.approx(d[up], rel=2e-6, abs=1e-6 * max(1.0, abs(d[up])))


def test_derivs_plummer_value(oracle):
    R = np.array([0.1, 0.2, -0.3])
    e2 = 0.01
    D, k = oracle.derivs(3, R, e2)
    d = _dict(D, k)
    s = (R * R).sum() + e2
    assert d[(0, 0, 0)] == pytest.approx(-s ** -0.5, rel=1e-15)
    assert d[(1, 0, 0)] == pytest.approx(R[0] * s ** -1.5, rel=1e-14)


def test_derivs_parity(oracle):
    # D^k(-R) = (-1)^{|k|} D^k(R): the property behind F_AB = -F_BA (Eq. 2)
    R = np.array([0.37, -0.21, 0.55])
    D1, k = oracle.derivs(5, R)
    D2, _ = oracle.derivs(5, -R)
    sg = np.array([(-1) ** int(sum(kk)) for kk in k])
    np.testing.assert_allclose(D2, sg * D1, rtol=1e-14, atol=0)
