"""GPU parity in the configuration the benchmark's headline figure is measured
in, and at the leaf sizes and softening lengths no other parity case reaches.

* cold collapse, N = 2^20 uniform in the unit sphere, Wendland eps = 0.005,
  p = 6, theta = 0.5, leaf 96 and leaf 128 (the two leaf sizes the tuner
  picks), built and evaluated with fmm_forces exactly as the benchmark times
  it: tree, permutation and both interaction lists bit-exact; FP64 forces and
  potentials within 1e-12 of the oracle on 256 seeded sinks plus every
  particle of two leaves holding more than 64 (the P2P kernel takes a leaf's
  sinks 64 at a time, so those leaves run its second pass); mixed precision
  within 2e-6 rms on the same sinks; the force gradient (fmm_forces_grad, the
  input of the fourth-order integrator of Sec. 4.1) on the same sinks against
  the oracle's per-sink gradient, FP64 within 1e-10 and mixed within 1e-5 rms
  of each tensor's size, its forces equal to those of fmm_forces bit for bit;
* a 20,000-particle sphere at leaf 128, compared element by element with the
  oracle FMM in both kernels and both precisions (every leaf of 65..128
  particles included);
* eps = 0 (no softening: the P2P kernel then excludes the self pair by its
  stream position instead of subtracting its potential term), both kernels,
  both precisions, leaf 16 and leaf 128.
"""
import numpy as np
import pytest

from conftest import gpu_available
from paper_1712_10116_amd import workloads as W

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

N = 1 << 20
EPS = 0.005


def _rel(a, ref):
    mag = np.sqrt((ref * ref).sum(axis=0))
    floor = 1e-6 * np.sqrt((mag * mag).mean())
    return np.sqrt(((a - ref) ** 2).sum(axis=0)) / np.maximum(mag, floor)


def _prel(p, ref):
    floor = 1e-6 * np.sqrt((ref * ref).mean())
    return np.abs(p - ref) / np.maximum(np.abs(ref), floor)


def _solve(pos, m, *, p, theta, eps, leaf, kernel, precision, export=False):
    import torch
    from paper_1712_10116_amd import fmm as F
    n = pos.shape[1]
    s = F.Solver(n, p_max=p, leaf_size=leaf, kernel=kernel, precision=precision)
    tp = torch.from_numpy(np.ascontiguousarray(pos)).cuda()
    tm = torch.from_numpy(np.ascontiguousarray(m)).cuda()
    a, pt = s.forces(tp, tm, eps=eps, theta=theta, p=p)
    ex = s.export_tree() if export else None
    info = s.tree_info()
    out = a.cpu().numpy(), pt.cpu().numpy(), ex, info
    s.close()
    return out


@pytest.fixture(scope="module", params=[96, 128])
def headline(request, oracle):
    leaf = request.param
    pos, _, m = W.uniform_sphere(N, seed=1001)
    t = oracle.Tree(pos, p=6, theta=0.5, eps=EPS, leaf_size=leaf, kernel=0)
    ref = t.export()
    cnt = ref["end"] - ref["begin"]
    big = np.flatnonzero((ref["is_leaf"] == 1) & (cnt > 64))
    assert big.size >= 2, "the workload must have leaves of more than 64 particles"
    pick = np.random.default_rng(78).choice(big, 2, replace=False)
    in_big = np.concatenate([ref["perm"][ref["begin"][c]:ref["end"][c]] for c in pick])
    rnd = np.random.default_rng(77).choice(N, 256, replace=False)
    sinks = np.unique(np.concatenate([rnd, in_big]))
    ra, rp, rg = t.evaluate_sinks_grad(m, sinks)
    return leaf, pos, m, t, ref, sinks, ra, rp, rg


def test_headline_tree_and_lists_bit_exact(headline):
    leaf, pos, m, t, ref, *_ = headline
    _, _, ex, info = _solve(pos, m, p=6, theta=0.5, eps=EPS, leaf=leaf, kernel=0, precision=1,
                            export=True)
    assert info["nodes"] == t.n_nodes and info["m2l"] == t.n_m2l and info["p2p"] == t.n_p2p
    for k in ("perm", "level", "prefix", "begin", "end", "is_leaf", "centre", "half", "box",
              "m2l", "p2p"):
        np.testing.assert_array_equal(ex[k], ref[k], err_msg=k)


@pytest.mark.parametrize("precision", [0, 1])
def test_headline_forces(headline, precision):
    leaf, pos, m, t, ref, sinks, ra, rp, _ = headline
    a, pt, _, _ = _solve(pos, m, p=6, theta=0.5, eps=EPS, leaf=leaf, kernel=0,
                         precision=precision)
    e = _rel(a[:, sinks], ra)
    ep = _prel(pt[sinks], rp)
    if precision == 0:
        assert e.max() < 1e-12 and ep.max() < 1e-12, (e.max(), ep.max())
    else:
        assert np.sqrt((e * e).mean()) < 2e-6 and np.sqrt((ep * ep).mean()) < 2e-6, (
            np.sqrt((e * e).mean()), np.sqrt((ep * ep).mean()))


@pytest.mark.parametrize("precision", [0, 1])
def test_headline_force_gradient(headline, precision):
    import torch
    from paper_1712_10116_amd import fmm as F
    leaf, pos, m, t, ref, sinks, ra, rp, rg = headline
    s = F.Solver(N, p_max=6, leaf_size=leaf, kernel=0, precision=precision)
    tp = torch.from_numpy(pos).cuda()
    tm = torch.from_numpy(m).cuda()
    a, pt, g = s.forces_grad(tp, tm, eps=EPS, theta=0.5, p=6)
    a2, pt2 = s.forces(tp, tm, eps=EPS, theta=0.5, p=6)
    torch.cuda.synchronize()
    assert torch.equal(a, a2) and torch.equal(pt, pt2)
    g = g.cpu().numpy()[:, sinks]
    s.close()
    e = np.sqrt(((g - rg) ** 2).sum(axis=0)) / np.sqrt((rg * rg).sum(axis=0))
    if precision == 0:
        assert e.max() < 1e-10, e.max()
    else:
        assert np.sqrt((e * e).mean()) < 1e-5, (np.sqrt((e * e).mean()), e.max())


@pytest.mark.parametrize("kernel", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_leaf128_every_particle(oracle, kernel, precision):
    pos, _, m = W.uniform_sphere(20000, seed=91)
    prm = dict(p=6, theta=0.5, eps=0.005, leaf_size=128, kernel=kernel)
    t = oracle.Tree(pos, **prm)
    ex = t.export()
    cnt = (ex["end"] - ex["begin"])[ex["is_leaf"] == 1]
    assert (cnt > 64).sum() >= 20 and cnt.max() <= 128
    ra, rp = t.evaluate(m)
    a, pt, gx, _ = _solve(pos, m, p=6, theta=0.5, eps=0.005, leaf=128, kernel=kernel,
                          precision=precision, export=True)
    for k in ("perm", "begin", "end", "m2l", "p2p"):
        np.testing.assert_array_equal(gx[k], ex[k], err_msg=k)
    e, ep = _rel(a, ra), _prel(pt, rp)
    if precision == 0:
        assert e.max() < 1e-12 and ep.max() < 1e-12, (e.max(), ep.max())
    else:
        assert np.sqrt((e * e).mean()) < 2e-6 and np.sqrt((ep * ep).mean()) < 2e-6, (
            np.sqrt((e * e).mean()), np.sqrt((ep * ep).mean()))


@pytest.mark.parametrize("leaf", [16, 128])
@pytest.mark.parametrize("kernel", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_unsoftened(oracle, leaf, kernel, precision):
    pos, _, m = W.plummer(12000, seed=92)
    prm = dict(p=5, theta=0.5, eps=0.0, leaf_size=leaf, kernel=kernel)
    ra, rp = oracle.fmm(pos, m, **prm)
    a, pt, _, _ = _solve(pos, m, p=5, theta=0.5, eps=0.0, leaf=leaf, kernel=kernel,
                         precision=precision)
    assert np.isfinite(a).all() and np.isfinite(pt).all()
    e, ep = _rel(a, ra), _prel(pt, rp)
    if precision == 0:
        assert e.max() < 1e-12 and ep.max() < 1e-12, (e.max(), ep.max())
    else:
        assert np.sqrt((e * e).mean()) < 2e-6 and np.sqrt((ep * ep).mean()) < 2e-6, (
            np.sqrt((e * e).mean()), np.sqrt((ep * ep).mean()))
