"""Pins of the total-acceleration timestep bound of Eq. (9) (Sec. 3.4) in the
oracle HHS (no GPU).

* the bound never binding (eta1 huge) changes nothing, bit for bit;
* |a|_tot is the magnitude of the acceleration due to all the mass: with one
  rung it equals |a| of numpy direct summation at the end-of-step positions;
* two equal masses at distance d: |a|_tot = m/d^2 (closed form), and with
  eta1 below eta the rung is the one that bound gives for that value;
* a binding bound only ever deepens rungs.
"""
import numpy as np

from paper_1712_10116_amd import workloads as W


def _direct_acc(pos, m, eps):
    d = pos[:, None, :] - pos[:, :, None]
    r2 = (d * d).sum(axis=0) + eps * eps
    np.fill_diagonal(r2, 1.0)
    g = r2 ** -1.5
    np.fill_diagonal(g, 0.0)
    return (d * (g * m[None, :])[None]).sum(axis=2)


def _run(oracle, pos, vel, m, steps, dt, **kw):
    H = oracle.HHSOracle(**kw)
    st = oracle.HHSState(pos, vel, m)
    H.init_forces(st)
    for _ in range(steps):
        H.step(st, dt)
    return st


KW = dict(p=4, theta=0.5, eps=0.01, leaf_size=16, eta=0.05, max_levels=5)


def test_loose_bound_changes_nothing(oracle):
    pos, vel, m = W.plummer(512, seed=31)
    a = _run(oracle, pos, vel, m, 2, 1.0 / 16, kernel=oracle.PLUMMER, **KW)
    b = _run(oracle, pos, vel, m, 2, 1.0 / 16, kernel=oracle.PLUMMER, eta1=1e30, **KW)
    assert len(np.unique(a.rung)) >= 2
    np.testing.assert_array_equal(a.rung, b.rung)
    np.testing.assert_array_equal(a.pos, b.pos)
    np.testing.assert_array_equal(a.vel, b.vel)
    assert a.force_calls == b.force_calls


def test_a_tot_is_full_acceleration(oracle):
    pos, vel, m = W.plummer(200, seed=32)
    eps = 0.05
    st = _run(oracle, pos, vel, m, 2, 1.0 / 64, p=3, theta=1e-6, eps=eps, leaf_size=8,
              kernel=oracle.PLUMMER, eta=0.05, max_levels=1, eta1=0.05)
    a = _direct_acc(st.pos, m, eps)
    np.testing.assert_allclose(st.a_tot, np.sqrt((a * a).sum(axis=0)), rtol=1e-12)


def test_two_body_rung_from_closed_form(oracle):
    d, mm, eps, dt_top = 0.5, 0.3, 1e-3, 1.0 / 8
    pos = np.array([[-d / 2, d / 2], [0.0, 0.0], [0.0, 0.0]])
    vel = np.zeros((3, 2))
    m = np.array([mm, mm])
    eta, eta1 = 20.0, 0.1
    H = oracle.HHSOracle(p=3, theta=1e-6, eps=eps, leaf_size=1, kernel=oracle.WENDLAND, eta=eta,
                         max_levels=8, eta1=eta1)
    st = oracle.HHSState(pos, vel, m)
    H.init_forces(st)
    a = mm / d ** 2                                   # Newtonian beyond the kernel radius
    np.testing.assert_allclose(st.a_tot, [a, a], rtol=1e-14)
    r_eta = next(k for k in range(8) if np.ldexp(dt_top, -k) ** 2 * a <= eta * eps)
    r_eta1 = next(k for k in range(8) if np.ldexp(dt_top, -k) ** 2 * a <= eta1 * eps)
    assert r_eta == 0 and r_eta1 == 4
    np.testing.assert_array_equal(H.rungs(st, np.arange(2), dt_top), [r_eta1, r_eta1])
    H0 = oracle.HHSOracle(p=3, theta=1e-6, eps=eps, leaf_size=1, kernel=oracle.WENDLAND,
                          eta=eta, max_levels=8)
    np.testing.assert_array_equal(H0.rungs(st, np.arange(2), dt_top), [r_eta, r_eta])


def test_binding_bound_deepens_rungs(oracle):
    pos, vel, m = W.plummer(1024, seed=33)
    kw = dict(KW, kernel=oracle.PLUMMER)
    H0 = oracle.HHSOracle(**kw)
    H1 = oracle.HHSOracle(eta1=0.005, **kw)
    st = oracle.HHSState(pos, vel, m)
    H1.init_forces(st)
    r0 = H0.rungs(st, np.arange(1024), 1.0 / 16)
    r1 = H1.rungs(st, np.arange(1024), 1.0 / 16)
    assert (r1 >= r0).all() and (r1 > r0).any()
    H1.step(st, 1.0 / 16)
    assert (st.a_tot > 0).all()
