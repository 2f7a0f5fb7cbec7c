"""The oracle's invariant sums (Sec. 3.2: momentum, angular momentum and
energy as accuracy monitors) pinned by closed forms: a ring of equal masses
in rigid rotation about its axis and moving as a whole."""
import numpy as np


def _ring(n, R, omega, V, X):
    ph = 2.0 * np.pi * np.arange(n) / n
    x = np.stack([R * np.cos(ph), R * np.sin(ph), np.zeros(n)])
    v = np.stack([-omega * R * np.sin(ph), omega * R * np.cos(ph), np.zeros(n)])
    return x + np.asarray(X)[:, None], v + np.asarray(V)[:, None]


def test_ring_closed_forms(oracle):
    n, M, R, om = 64, 3.0, 2.0, 0.7
    V, X = np.array([0.3, -0.2, 0.1]), np.array([1.0, 2.0, -0.5])
    pos, vel = _ring(n, R, om, V, X)
    m = np.full(n, M / n)
    # acceleration of the rigid rotation (centripetal) and a potential of -1 each
    acc = -(om * om) * (pos - X[:, None])
    pot = np.full(n, -1.0)
    inv = oracle.invariants(pos, vel, m, acc=acc, pot=pot)
    np.testing.assert_allclose(inv["P"], M * V, rtol=1e-14, atol=1e-15)
    # L = M X x V (centre of mass) + M R^2 omega z (spin about the centre)
    L = M * np.cross(X, V) + np.array([0.0, 0.0, M * R * R * om])
    np.testing.assert_allclose(inv["L"], L, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(inv["T"], 0.5 * M * (R * R * om * om + V @ V), rtol=1e-14)
    np.testing.assert_allclose(inv["W"], -0.5 * M, rtol=1e-14)
    np.testing.assert_allclose(inv["F"], 0.0, atol=1e-14)
    np.testing.assert_allclose(inv["Fabs"], M * om * om * R, rtol=1e-14)
