"""Comoving drift and kick factors (Sec. 3.5, Eqs. 10-11) (no GPU: host code).

Oracle pins against closed forms: Einstein-de Sitter (H = h0 a^-3/2), empty
open (H = h0/a) and de Sitter (H = h0).  The library's lookup table against
the oracle for a flat LambdaCDM cosmology and the three special cases, over
steps inside one grid interval and across many, forward and backward; range
and parameter errors.
"""
import math

import numpy as np
import pytest

H0 = 0.1


def _closed(kind, a0, a1):
    if kind == "eds":       # a ~ t^(2/3)
        return (2 / H0) * (a0 ** -0.5 - a1 ** -0.5), (2 / H0) * (a1 ** 0.5 - a0 ** 0.5)
    if kind == "milne":     # a ~ t
        return (1 / a0 - 1 / a1) / H0, math.log(a1 / a0) / H0
    if kind == "desitter":  # a ~ e^(h0 t)
        return (a0 ** -2 - a1 ** -2) / (2 * H0), (1 / a0 - 1 / a1) / H0
    raise ValueError(kind)


COSMO = {"eds": (1.0, 0.0), "milne": (0.0, 0.0), "desitter": (0.0, 1.0),
         "lcdm": (0.3, 0.7)}
STEPS = [(0.02, 0.0201), (0.05, 0.9), (0.3, 0.31), (0.999, 0.2), (0.01, 1.0)]


@pytest.mark.parametrize("kind", ["eds", "milne", "desitter"])
def test_oracle_closed_forms(oracle, kind):
    om, ol = COSMO[kind]
    for a0, a1 in STEPS:
        d, k = oracle.cosmo_factors(a0, a1, omega_m=om, omega_l=ol, h0=H0)
        cd, ck = _closed(kind, a0, a1)
        assert abs(d - cd) <= 1e-11 * abs(cd) and abs(k - ck) <= 1e-11 * abs(ck), (a0, a1)


@pytest.mark.parametrize("kind", ["eds", "milne", "desitter", "lcdm"])
def test_table_matches_oracle(oracle, kind):
    from paper_1712_10116_amd import fmm as F
    om, ol = COSMO[kind]
    tab = F.Cosmology(omega_m=om, omega_l=ol, h0=H0, a_min=0.01, a_max=1.0, n=1000)
    for a0, a1 in STEPS:
        d, k = tab.factors(a0, a1)
        od, ok = oracle.cosmo_factors(a0, a1, omega_m=om, omega_l=ol, h0=H0)
        assert abs(d - od) <= 1e-12 * abs(od) and abs(k - ok) <= 1e-12 * abs(ok), (a0, a1)
    assert tab.factors(0.5, 0.5) == (0.0, 0.0)
    tab.close()


def test_table_errors():
    from paper_1712_10116_amd import fmm as F
    tab = F.Cosmology(omega_m=0.3, omega_l=0.7, h0=H0, a_min=0.1, a_max=1.0, n=64)
    with pytest.raises(F.FMMError):
        tab.factors(0.05, 0.5)           # below the table
    with pytest.raises(F.FMMError):
        tab.factors(0.5, 1.5)            # above it
    tab.close()
    with pytest.raises(F.FMMError):
        F.Cosmology(omega_m=0.3, omega_l=0.7, h0=H0, a_min=1.0, a_max=0.5)
    with pytest.raises(F.FMMError):      # closed universe that recollapses inside the range
        F.Cosmology(omega_m=5.0, omega_l=0.0, h0=H0, a_min=0.1, a_max=2.0)


def _direct_acc(pos, m, eps):
    d = pos[:, None, :] - pos[:, :, None]
    r2 = (d * d).sum(axis=0) + eps * eps
    np.fill_diagonal(r2, 1.0)
    g = r2 ** -1.5
    np.fill_diagonal(g, 0.0)
    return (d * (g * m[None, :])[None]).sum(axis=2)


def test_oracle_comoving_single_rung_is_leapfrog(oracle):
    """One rung, Einstein-de Sitter: the comoving HHS is the textbook
    kick-drift-kick with the closed-form factors of its own sub-intervals."""
    from paper_1712_10116_amd import workloads as W
    pos, vel, m = W.plummer(150, seed=51)
    eps, dx = 0.05, 0.05                         # steps of 0.05 in ln a from a = 0.2
    cos = dict(omega_m=1.0, omega_l=0.0, h0=H0)
    H = oracle.HHSOracle(p=3, theta=1e-6, eps=eps, leaf_size=8, kernel=oracle.PLUMMER,
                         eta=0.05, max_levels=1, cosmo=cos)
    st = oracle.HHSState(pos, vel, m)
    st.t = math.log(0.2)
    H.init_forces(st)
    x, p, t = pos.copy(), vel.copy(), math.log(0.2)
    for _ in range(3):
        H.step(st, dx)
        a0, ah, a1 = math.exp(t), math.exp(t + dx / 2), math.exp(t + dx)
        p = p + _closed("eds", a0, ah)[1] * _direct_acc(x, m, eps)
        x = x + _closed("eds", a0, a1)[0] * p
        p = p + _closed("eds", ah, a1)[1] * _direct_acc(x, m, eps)
        t += dx
    assert abs(st.t - t) < 1e-15
    np.testing.assert_allclose(st.pos, x, rtol=0, atol=1e-11)
    np.testing.assert_allclose(st.vel, p, rtol=0, atol=1e-11)


def test_oracle_comoving_momentum_conserved(oracle):
    from paper_1712_10116_amd import workloads as W
    pos, vel, m = W.plummer(1024, seed=52)
    H = oracle.HHSOracle(p=4, theta=0.5, eps=0.01, leaf_size=16, kernel=oracle.PLUMMER,
                         eta=0.05, max_levels=4, cosmo=dict(omega_m=0.3, omega_l=0.7, h0=1.0))
    st = oracle.HHSState(pos, vel, m)
    st.t = math.log(0.5)
    H.init_forces(st)
    P0 = (m * vel).sum(axis=1)
    H.step(st, 1.0 / 16)
    assert len(np.unique(st.rung)) >= 2
    scale = (m * np.sqrt((vel * vel).sum(axis=0))).sum()
    assert np.abs((m * st.vel).sum(axis=1) - P0).max() / scale < 1e-14
    assert np.abs(st.pos - pos).max() > 1e-4
