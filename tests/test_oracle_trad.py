"""Pins of the oracle's individual-timestep integrator (Sec. 2.3) (no GPU).

* one rung only, or every particle on one rung: the scheme is the textbook
  kick-drift-kick leapfrog with dt_top / 2^rung, checked against a leapfrog
  written here with numpy direct-summation forces;
* a massless particle on rung 3 orbiting a heavy mass that coasts on rung 0:
  the light particle follows a leapfrog in the field of a point mass that
  stays where its last step ended (x0) until the top step ends -- inactive
  positions are not synchronised -- and the heavy mass moves by v dt_top;
* solver calls: 1 + 2^R per top step, R the deepest rung present;
* total momentum is not conserved once rungs differ (the paper's contrast with
  HHS, Sec. 3.2), while HHS on the same system conserves it to round-off.
"""
import numpy as np

from paper_1712_10116_amd import workloads as W


def _direct_acc(pos, m, eps):
    d = pos[:, None, :] - pos[:, :, None]          # x_j - x_i  [axis, i, j]
    r2 = (d * d).sum(axis=0) + eps * eps
    np.fill_diagonal(r2, 1.0)
    g = r2 ** -1.5
    np.fill_diagonal(g, 0.0)
    return (d * (g * m[None, :])[None]).sum(axis=2)


def _leapfrog(x, v, m, eps, dt, steps):
    for _ in range(steps):
        v = v + 0.5 * dt * _direct_acc(x, m, eps)
        x = x + dt * v
        v = v + 0.5 * dt * _direct_acc(x, m, eps)
    return x, v


def _trad(oracle, pos, vel, m, *, eps, eta, max_levels, kernel, theta=1e-6, p=3, leaf=8):
    T = oracle.TradOracle(p=p, theta=theta, eps=eps, leaf_size=leaf, kernel=kernel, eta=eta,
                          max_levels=max_levels)
    return T, oracle.HHSState(pos, vel, m)


def test_single_rung_is_leapfrog(oracle):
    pos, vel, m = W.plummer(200, seed=21)
    eps, dt = 0.05, 1.0 / 64
    T, st = _trad(oracle, pos, vel, m, eps=eps, eta=0.05, max_levels=1, kernel=oracle.PLUMMER)
    for _ in range(3):
        T.step(st, dt)
    x, v = _leapfrog(pos.copy(), vel.copy(), m, eps, dt, 3)
    assert st.force_calls == 3 * 2
    np.testing.assert_allclose(st.pos, x, rtol=0, atol=1e-12)
    np.testing.assert_allclose(st.vel, v, rtol=0, atol=1e-12)


def test_common_deep_rung_is_leapfrog(oracle):
    # eta so small that every particle is clamped to the deepest rung, 2
    pos, vel, m = W.plummer(150, seed=22)
    eps, dt = 0.05, 1.0 / 16
    T, st = _trad(oracle, pos, vel, m, eps=eps, eta=1e-12, max_levels=3, kernel=oracle.PLUMMER)
    T.step(st, dt)
    assert (st.rung == 2).all()
    assert st.force_calls == 1 + 4
    x, v = _leapfrog(pos.copy(), vel.copy(), m, eps, dt / 4, 4)
    np.testing.assert_allclose(st.pos, x, rtol=0, atol=1e-12)
    np.testing.assert_allclose(st.vel, v, rtol=0, atol=1e-12)


def test_unsynchronised_source_position(oracle):
    # heavy mass M = 1 coasting at velocity u (no force reaches it: its
    # companion is massless); the companion on a near-circular orbit of
    # radius 1.  Wendland kernel with eps far below the separation: the
    # force is exactly Newtonian.
    eps, eta, dt_top, steps = 1e-3, 0.4, 1.0 / 8, 2
    u = np.array([0.3, -0.2, 0.1])
    pos = np.array([[0.0, 1.0], [0.0, 0.0], [0.0, 0.0]])
    vel = np.array([[u[0], u[0]], [u[1], u[1] + 1.0], [u[2], u[2]]])
    m = np.array([1.0, 0.0])
    T, st = _trad(oracle, pos, vel, m, eps=eps, eta=eta, max_levels=6, kernel=oracle.WENDLAND,
                  leaf=1)
    # rung of the light particle: smallest r with (dt_top 2^-r)^2 |a| <= eta eps, |a| = 1
    r = next(k for k in range(6) if np.ldexp(dt_top, -k) ** 2 * 1.0 <= eta * eps)
    assert r == 3
    ticks = 1 << r
    h = dt_top / ticks
    xm, vm = pos[:, 0].copy(), vel[:, 0].copy()
    x, v = pos[:, 1].copy(), vel[:, 1].copy()

    def pull(at, src):
        d = src - at
        return d / np.sqrt(d @ d) ** 3

    for _ in range(steps):
        T.step(st, dt_top)
        assert list(st.rung) == [0, r]
        v = v + 0.5 * h * pull(x, xm)
        for j in range(ticks):
            x = x + h * v
            src = xm + dt_top * vm if j == ticks - 1 else xm   # M drifts only at the end
            a = pull(x, src)
            v = v + 0.5 * h * a
            if j < ticks - 1:
                v = v + 0.5 * h * a
        xm = xm + dt_top * vm
    assert st.force_calls == steps * (1 + ticks)
    np.testing.assert_allclose(st.pos[:, 0], xm, rtol=0, atol=1e-14)
    np.testing.assert_array_equal(st.vel[:, 0], vel[:, 0])
    np.testing.assert_allclose(st.pos[:, 1], x, rtol=0, atol=1e-12)
    np.testing.assert_allclose(st.vel[:, 1], v, rtol=0, atol=1e-12)


def test_momentum_drift_against_hhs(oracle):
    pos, vel, m = W.plummer(1024, seed=23)
    kw = dict(p=4, theta=0.5, eps=0.01, leaf_size=16, kernel=oracle.PLUMMER, eta=0.05,
              max_levels=4)
    dt = 1.0 / 16
    scale = (m * np.sqrt((vel * vel).sum(axis=0))).sum()
    P0 = (m * vel).sum(axis=1)
    T = oracle.TradOracle(**kw)
    st = oracle.HHSState(pos, vel, m)
    T.step(st, dt)
    assert len(np.unique(st.rung)) >= 2
    assert st.force_calls == 1 + (1 << int(st.rung.max()))
    dp_trad = np.abs((m * st.vel).sum(axis=1) - P0).max() / scale
    H = oracle.HHSOracle(**kw)
    sh = oracle.HHSState(pos, vel, m)
    H.init_forces(sh)
    H.step(sh, dt)
    dp_hhs = np.abs((m * sh.vel).sum(axis=1) - P0).max() / scale
    assert dp_hhs < 1e-14
    assert dp_trad > 1e-9
