"""Pins of the oracle's force gradient d a_i / d x_i (the tidal tensor that the
Chin integrator of Sec. 4.1 needs from the FMM) (no GPU).

* a massless particle at x from a unit point mass: (3 x x^T - r^2 I) / r^5
  (closed form), the mass itself feels nothing;
* theta -> 0 (every pair by P2P): the tensor equals central finite differences
  of numpy direct-summation accelerations with respect to the sink's own
  position, for the Plummer kernel and for Wendland pairs inside the kernel
  radius (the interior polynomial's derivative);
* Newtonian pairs only: the tensor is traceless (Laplace);
* at theta = 0.5 the FMM tensor converges to the direct one as p grows.
"""
import numpy as np

from paper_1712_10116_amd import workloads as W

COMP = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def _direct_acc_i(pos, m, i, xi, kernel, eps):
    """Acceleration of particle i placed at xi (numpy, plain definition)."""
    d = pos - xi[:, None]
    r2 = (d * d).sum(axis=0)
    r2[i] = 1.0
    r = np.sqrt(r2)
    if kernel == 1:                                     # Plummer
        g = (r2 + eps * eps) ** -1.5
    else:                                               # Wendland C2, Eq. (8)
        u = r / eps
        inside = 21 * u**5 - 90 * u**4 + 140 * u**3 - 84 * u**2 + 14
        g = np.where(r >= eps, 1.0 / (r2 * r), inside / eps**3)
    g[i] = 0.0
    return (d * (m * g)[None]).sum(axis=1)


def _fd_grad(pos, m, i, kernel, eps, h):
    out = np.zeros((3, 3))
    for b in range(3):
        e = np.zeros(3)
        e[b] = h
        out[:, b] = (_direct_acc_i(pos, m, i, pos[:, i] + e, kernel, eps)
                     - _direct_acc_i(pos, m, i, pos[:, i] - e, kernel, eps)) / (2 * h)
    return out


def _tensor(grad, i):
    T = np.zeros((3, 3))
    for c, (a, b) in enumerate(COMP):
        T[a, b] = T[b, a] = grad[c, i]
    return T


def _grad(oracle, pos, m, **kw):
    t = oracle.Tree(pos, None, **kw)
    return t.evaluate_grad(m)


def test_point_mass_closed_form(oracle):
    x = np.array([0.3, -0.4, 0.5])
    pos = np.array([[0.0, x[0]], [0.0, x[1]], [0.0, x[2]]])
    m = np.array([1.0, 0.0])
    _, _, g = _grad(oracle, pos, m, p=3, theta=1e-6, eps=1e-3, leaf_size=1,
                    kernel=oracle.WENDLAND)
    r2 = x @ x
    exact = (3 * np.outer(x, x) - r2 * np.eye(3)) / r2 ** 2.5
    np.testing.assert_allclose(_tensor(g, 1), exact, rtol=1e-13, atol=1e-13)
    assert (g[:, 0] == 0).all()


def test_direct_limit_equals_finite_differences(oracle):
    pos, _, m = W.plummer(300, seed=41)
    d = pos[:, :, None] - pos[:, None, :]
    r = np.sqrt((d * d).sum(axis=0))
    inside = (r < 0.3).sum(axis=1) - 1            # neighbours within eps = 0.3
    crowded = [int(i) for i in np.argsort(-inside)[:3]]
    assert inside[crowded].min() >= 3             # interior Wendland pairs are exercised
    for kernel, eps in ((oracle.PLUMMER, 0.05), (oracle.WENDLAND, 0.3)):
        _, _, g = _grad(oracle, pos, m, p=3, theta=1e-6, eps=eps, leaf_size=8, kernel=kernel)
        for i in [0, 150, 299] + crowded:
            fd = _fd_grad(pos, m, i, kernel, eps, 1e-5)
            T = _tensor(g, i)
            np.testing.assert_allclose(T, fd, rtol=0, atol=1e-6 * np.abs(fd).max())


def test_traceless_outside_the_kernel(oracle):
    pos, _, m = W.uniform_sphere(400, seed=42)
    _, _, g = _grad(oracle, pos, m, p=3, theta=1e-6, eps=1e-6, leaf_size=8,
                    kernel=oracle.WENDLAND)
    tr = g[0] + g[1] + g[2]
    assert np.abs(tr).max() < 1e-9 * np.abs(g[:3]).max()


def test_converges_in_p(oracle):
    pos, _, m = W.plummer(2000, seed=43)
    kw = dict(eps=0.01, leaf_size=16, kernel=oracle.PLUMMER)
    _, _, ref = _grad(oracle, pos, m, p=3, theta=1e-6, **kw)
    errs = []
    for p in (2, 4, 6, 8):
        _, _, g = _grad(oracle, pos, m, p=p, theta=0.5, **kw)
        errs.append(np.sqrt(((g - ref) ** 2).sum() / (ref ** 2).sum()))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-3, errs


def test_sampled_sinks_equal_full_evaluation(oracle):
    """The per-sink evaluation (path M2L/L2L, the leaf's partners) gives the
    force gradient of the full evaluation, and the same forces as the plain
    per-sink call; a dropped Hessian term or a wrong pair sign fails it."""
    for kernel, eps in ((oracle.WENDLAND, 0.05), (oracle.PLUMMER, 0.01)):
        pos, _, m = W.uniform_sphere(3000, seed=44)
        m = m * np.random.default_rng(45).uniform(0.5, 1.5, m.size)
        t = oracle.Tree(pos, None, p=5, theta=0.5, eps=eps, leaf_size=24, kernel=kernel)
        _, _, full = t.evaluate_grad(m)
        sinks = np.random.default_rng(46).choice(m.size, 200, replace=False)
        a, pt, g = t.evaluate_sinks_grad(m, sinks)
        a2, pt2 = t.evaluate_sinks(m, sinks)
        assert np.array_equal(a, a2) and np.array_equal(pt, pt2)
        ref = full[:, sinks]
        scale = np.sqrt((ref * ref).sum(axis=0))
        assert (np.sqrt(((g - ref) ** 2).sum(axis=0)) / scale).max() < 1e-12
