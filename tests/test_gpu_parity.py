"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

* tree, permutation, cell geometry and both interaction lists: bit-exact;
* FP64 forces and potentials: within 1e-12 relative of the same-parameter
  oracle FMM (per particle, floor 1e-6 of the rms magnitude);
* mixed precision: within 2e-6 rms relative;
* total momentum: <= 1e-13 relative in FP64, <= 1e-6 in mixed precision,
  also across a masked (kickS2F) / unmasked (kickFS2S) pair of calls;
* edge cases: empty, one and two particles, coincident particles, leaf size
  1 and 64, active subsets in random order, zero masses;
* run-to-run bit identity.
"""
import numpy as np
import pytest

from conftest import gpu_available
from paper_1712_10116_amd import workloads as W

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _torch():
    import torch
    return torch


def _F():
    from paper_1712_10116_amd import fmm as F
    return F


def rel_err(a, ref):
    mag = np.sqrt((ref * ref).sum(axis=0))
    floor = 1e-6 * np.sqrt((mag * mag).mean()) if mag.size else 1.0
    return np.sqrt(((a - ref) ** 2).sum(axis=0)) / np.maximum(mag, floor)


def pot_err(p, ref):
    floor = 1e-6 * np.sqrt((ref * ref).mean()) if ref.size else 1.0
    return np.abs(p - ref) / np.maximum(np.abs(ref), floor)


def gpu_solve(pos, mass, active=None, *, p, theta, eps, leaf_size, kernel, precision,
              export=False):
    torch, F = _torch(), _F()
    dev = torch.device("cuda:0")
    n = pos.shape[1] if active is None else len(active)
    s = F.Solver(max(n, 1), p_max=max(p, 1), leaf_size=leaf_size, kernel=kernel,
                 precision=precision)
    tp = torch.from_numpy(np.ascontiguousarray(pos)).to(dev)
    tm = torch.from_numpy(np.ascontiguousarray(mass)).to(dev)
    ta = None if active is None else torch.from_numpy(np.asarray(active, dtype=np.int32)).to(dev)
    s.build(tp, ta, eps=eps, theta=theta)
    ex = s.export_tree() if export else None
    info = s.tree_info()
    a, pt = s.evaluate(tp, tm, ta, p=p)
    torch.cuda.synchronize()
    out = a.cpu().numpy(), pt.cpu().numpy(), ex, info
    s.close()
    return out


TREE_CASES = [
    # (label, generator, n, leaf, theta, eps, active)
    ("plummer4096", lambda: W.config(0, n=4096), 4096, 16, 0.5, 0.01, None),
    ("sphere5000", lambda: W.config(1, n=5000), 5000, 16, 0.5, 0.005, None),
    ("disk6001", lambda: W.disk_galaxy(6001, seed=7), 6001, 8, 0.4, 0.02, None),
    ("zoom7003", lambda: W.clustered_zoom(7003, seed=8, n_halos=40), 7003, 16, 0.4, 0.001, None),
    ("leaf1", lambda: W.config(0, n=300), 300, 1, 0.5, 0.01, None),
    ("leaf64", lambda: W.config(1, n=3000), 3000, 64, 0.3, 0.005, None),
    ("subset", lambda: W.config(1, n=5000), 5000, 16, 0.5, 0.005, "random"),
]


def _case(label):
    for c in TREE_CASES:
        if c[0] == label:
            return c
    raise KeyError(label)


def _inputs(case):
    label, gen, n, leaf, theta, eps, act = case
    pos, _, m = gen()
    active = None
    if act == "random":
        active = np.random.default_rng(11).permutation(pos.shape[1])[:3001].astype(np.int32)
    return pos, m, active, leaf, theta, eps


@pytest.mark.parametrize("label", [c[0] for c in TREE_CASES])
def test_tree_and_lists_bit_exact(oracle, label):
    F = _F()
    pos, m, active, leaf, theta, eps = _inputs(_case(label))
    t = oracle.Tree(pos, active, p=4, theta=theta, eps=eps, leaf_size=leaf, kernel=0)
    ref = t.export()
    _, _, ex, info = gpu_solve(pos, m, active, p=4, theta=theta, eps=eps, leaf_size=leaf,
                               kernel=F.WENDLAND, precision=F.FP64, export=True)
    assert info["nodes"] == t.n_nodes and info["depth"] == t.depth
    assert info["m2l"] == t.n_m2l and info["p2p"] == t.n_p2p
    for k in ("perm", "level", "prefix", "begin", "end", "is_leaf", "m2l", "p2p"):
        np.testing.assert_array_equal(ex[k], ref[k], err_msg=k)
    for k in ("centre", "half", "box"):
        np.testing.assert_array_equal(ex[k], ref[k], err_msg=k)


@pytest.mark.parametrize("label", ["plummer4096", "sphere5000", "zoom7003", "subset", "leaf64"])
@pytest.mark.parametrize("kernel", [0, 1])
def test_fp64_forces_match_oracle(oracle, label, kernel):
    F = _F()
    pos, m, active, leaf, theta, eps = _inputs(_case(label))
    p = 4
    ra, rp = oracle.fmm(pos, m, active, p=p, theta=theta, eps=eps, leaf_size=leaf, kernel=kernel)
    a, pt, _, _ = gpu_solve(pos, m, active, p=p, theta=theta, eps=eps, leaf_size=leaf,
                            kernel=kernel, precision=F.FP64)
    assert rel_err(a, ra).max() < 1e-12
    assert pot_err(pt, rp).max() < 1e-12


@pytest.mark.parametrize("p", [1, 2, 3, 5, 6])
def test_fp64_every_order(oracle, p):
    F = _F()
    pos, _, m = W.config(0, n=2500)
    ra, rp = oracle.fmm(pos, m, p=p, theta=0.45, eps=0.01, leaf_size=16, kernel=1)
    a, pt, _, _ = gpu_solve(pos, m, p=p, theta=0.45, eps=0.01, leaf_size=16, kernel=1,
                            precision=F.FP64)
    assert rel_err(a, ra).max() < 1e-12
    assert pot_err(pt, rp).max() < 1e-12


@pytest.mark.parametrize("label", ["plummer4096", "sphere5000", "zoom7003", "subset"])
@pytest.mark.parametrize("kernel", [0, 1])
@pytest.mark.parametrize("p", [4, 6])
def test_mixed_forces_match_oracle(oracle, label, kernel, p):
    F = _F()
    pos, m, active, leaf, theta, eps = _inputs(_case(label))
    ra, rp = oracle.fmm(pos, m, active, p=p, theta=theta, eps=eps, leaf_size=leaf, kernel=kernel)
    a, pt, _, _ = gpu_solve(pos, m, active, p=p, theta=theta, eps=eps, leaf_size=leaf,
                            kernel=kernel, precision=F.MIXED)
    e = rel_err(a, ra)
    assert np.sqrt((e * e).mean()) < 2e-6, (np.sqrt((e * e).mean()), e.max())
    ep = pot_err(pt, rp)
    assert np.sqrt((ep * ep).mean()) < 2e-6


@pytest.mark.parametrize("precision,tol", [(0, 1e-13), (1, 1e-6)])
def test_momentum_and_cross_call(oracle, precision, tol):
    torch, F = _torch(), _F()
    pos, _, m = W.config(1, n=20000)
    dev = torch.device("cuda:0")
    s = F.Solver(20000, p_max=4, leaf_size=16, kernel=F.WENDLAND, precision=precision)
    tp = torch.from_numpy(pos).to(dev)
    tm = torch.from_numpy(m).to(dev)
    a, _ = s.forces(tp, tm, eps=0.005, theta=0.5, p=4)
    inv = s.invariants(mass=tm, acc=a)
    assert np.abs(inv["F"]).max() / inv["Fabs"] < tol
    # kickS2F / kickFS2S pair on one tree
    fast = np.random.default_rng(2).uniform(size=20000) < 0.3
    mm = m.copy(); mm[fast] = 0.0
    s.build(tp, eps=0.005, theta=0.5)
    a1, _ = s.evaluate(tp, torch.from_numpy(mm).to(dev), p=4)
    a2, _ = s.evaluate(tp, tm, p=4)
    torch.cuda.synchronize()
    a1, a2 = a1.cpu().numpy(), a2.cpu().numpy()
    tot = (m[fast] * a1[:, fast]).sum(axis=1) + (m[~fast] * a2[:, ~fast]).sum(axis=1)
    assert np.abs(tot).max() / (m * np.sqrt((a2 ** 2).sum(axis=0))).sum() < tol
    s.close()


def test_edge_cases(oracle):
    F = _F()
    prm = dict(p=4, theta=0.5, eps=0.01, leaf_size=4, kernel=1)
    # one particle
    a, pt, ex, info = gpu_solve(np.zeros((3, 1)), np.ones(1), precision=F.FP64, export=True, **prm)
    assert (a == 0).all() and (pt == 0).all() and info["nodes"] == 1
    # two particles
    pos = np.array([[0.0, 0.3], [0.0, 0.4], [0.0, 0.0]])
    ra, rp = oracle.fmm(pos, np.array([1.0, 2.0]), **prm)
    a, pt, _, _ = gpu_solve(pos, np.array([1.0, 2.0]), precision=F.FP64, **prm)
    np.testing.assert_allclose(a, ra, rtol=1e-14)
    # coincident particles (depth-21 leaf) plus a cloud, zero masses included
    rng = np.random.default_rng(3)
    pos = np.concatenate([np.full((3, 40), 0.125), rng.uniform(size=(3, 500))], axis=1)
    m = rng.uniform(size=540); m[::7] = 0.0
    t = oracle.Tree(pos, **prm)
    ref = t.export()
    ra, rp = t.evaluate(m)
    a, pt, ex, info = gpu_solve(pos, m, precision=F.FP64, export=True, **prm)
    assert info["depth"] == 21
    for k in ("perm", "begin", "end", "level", "m2l", "p2p"):
        np.testing.assert_array_equal(ex[k], ref[k])
    assert rel_err(a, ra).max() < 1e-12
    # empty active set
    torch = _torch()
    s = F.Solver(10, p_max=4, leaf_size=4, kernel=1, precision=F.FP64)
    tp = torch.zeros((3, 10), dtype=torch.float64, device="cuda:0")
    ta = torch.zeros((0,), dtype=torch.int32, device="cuda:0")
    acc, pot = s.forces(tp, torch.ones(10, dtype=torch.float64, device="cuda:0"), ta, eps=0.01,
                        theta=0.5, p=4)
    assert acc.shape == (3, 0)
    assert s.tree_info()["nodes"] == 1  # one empty root cell per system
    s.close()


def test_errors_reported(oracle):
    torch, F = _torch(), _F()
    s = F.Solver(100, p_max=4, leaf_size=8, kernel=0, precision=F.FP64)
    tp = torch.zeros((3, 100), dtype=torch.float64, device="cuda:0")
    tp[0, 5] = float("nan")
    with pytest.raises(F.FMMError) as ei:
        s.build(tp, eps=0.01, theta=0.5)
    assert ei.value.status == F.FMM_ENONFINITE
    tp[0, 5] = 0.0
    with pytest.raises(F.FMMError) as ei:
        s.evaluate(tp, torch.ones(100, dtype=torch.float64, device="cuda:0"), p=4)
    assert ei.value.status == F.FMM_ESTALE
    s.build(tp, eps=0.01, theta=0.5)
    with pytest.raises(F.FMMError):
        s.evaluate(tp, torch.ones(100, dtype=torch.float64, device="cuda:0"), p=7)
    s.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_run_to_run_bit_identical(precision):
    F = _F()
    pos, _, m = W.config(1, n=30000)
    r1 = gpu_solve(pos, m, p=4, theta=0.5, eps=0.005, leaf_size=16, kernel=0, precision=precision)
    r2 = gpu_solve(pos, m, p=4, theta=0.5, eps=0.005, leaf_size=16, kernel=0, precision=precision)
    assert np.array_equal(r1[0], r2[0]) and np.array_equal(r1[1], r2[1])


@pytest.mark.parametrize("label", ["plummer4096", "subset", "zoom7003", "leaf1", "leaf64"])
@pytest.mark.parametrize("precision", [0, 1])
def test_small_and_general_paths_identical(label, precision):
    """Batches of at most 8192 particles are built and walked by one workgroup
    each; forcing the multi-workgroup path gives the same tree, lists and
    forces bit for bit."""
    torch, F = _torch(), _F()
    pos, m, active, leaf, theta, eps = _inputs(_case(label))
    out = []
    for small in (True, False):
        n = pos.shape[1] if active is None else len(active)
        s = F.Solver(n, p_max=4, leaf_size=leaf, kernel=F.WENDLAND, precision=precision)
        s.set_small_path(2 if small else False)
        tp = torch.from_numpy(np.ascontiguousarray(pos)).cuda()
        tm = torch.from_numpy(np.ascontiguousarray(m)).cuda()
        ta = None if active is None else torch.from_numpy(active).cuda()
        s.build(tp, ta, eps=eps, theta=theta)
        ex = s.export_tree()
        a, pt = s.evaluate(tp, tm, ta, p=4)
        torch.cuda.synchronize()
        out.append((ex, a.cpu().numpy(), pt.cpu().numpy(), s.tree_info()))
        s.close()
    (e1, a1, p1, i1), (e2, a2, p2, i2) = out
    assert i1 == i2
    for k in e1:
        np.testing.assert_array_equal(e1[k], e2[k], err_msg=k)
    assert np.array_equal(a1, a2) and np.array_equal(p1, p2)


def test_level_prediction_identical():
    """Builds that queue tree and walk for the split depth of recent builds
    (one readback) give the same trees, lists and forces as the classic
    sequence: first build (no history), a deeper system after a shallow one
    (prediction too shallow: redone), a shallow one after a deep one (extra
    empty levels), and a repeat."""
    torch, F = _torch(), _F()
    seq = [W.uniform_sphere(30000, seed=41), W.plummer(30000, seed=42),
           W.uniform_sphere(20000, seed=43), W.uniform_sphere(20000, seed=43)]
    kw = dict(p_max=4, leaf_size=16, kernel=F.WENDLAND, precision=1)
    pred = F.Solver(30000, **kw)
    pred.set_level_prediction(True)
    for k, (pos, _, m) in enumerate(seq):
        tp = torch.from_numpy(np.ascontiguousarray(pos)).cuda()
        tm = torch.from_numpy(np.ascontiguousarray(m)).cuda()
        out = []
        for s in (pred, None):
            own = s is None
            if own:
                s = F.Solver(30000, **kw)
                s.set_level_prediction(False)
            s.build(tp, eps=0.01, theta=0.5)
            ex = s.export_tree()
            a, pt = s.evaluate(tp, tm, p=4)
            torch.cuda.synchronize()
            out.append((ex, a.cpu().numpy(), pt.cpu().numpy(), s.tree_info()))
            if own:
                s.close()
        (e1, a1, p1, i1), (e2, a2, p2, i2) = out
        assert i1 == i2, k
        for key in e1:
            np.testing.assert_array_equal(e1[key], e2[key], err_msg=f"{k} {key}")
        assert np.array_equal(a1, a2) and np.array_equal(p1, p2), k
    pred.close()


def test_fused_forces_identical():
    """forces() on a context with recent builds queues the evaluation behind
    the walk before the tree header is read; the result equals a classic
    build + evaluate bit for bit, also when the tree needs more levels than
    predicted, when the lists outgrow their workspace (theta lowered) and on
    a repeat."""
    torch, F = _torch(), _F()
    seq = [(W.uniform_sphere(30000, seed=51), 0.5), (W.uniform_sphere(30000, seed=52), 0.5),
           (W.plummer(30000, seed=53), 0.5), (W.plummer(30000, seed=53), 0.25),
           (W.plummer(30000, seed=53), 0.25)]
    for precision in (0, 1):
        kw = dict(p_max=4, leaf_size=16, kernel=F.WENDLAND, precision=precision)
        fused = F.Solver(30000, **kw)
        fused.set_level_prediction(True)
        for k, ((pos, _, m), theta) in enumerate(seq):
            tp = torch.from_numpy(np.ascontiguousarray(pos)).cuda()
            tm = torch.from_numpy(np.ascontiguousarray(m)).cuda()
            a1, p1 = fused.forces(tp, tm, eps=0.01, theta=theta, p=4)
            i1 = fused.tree_info()
            ref = F.Solver(30000, **kw)
            ref.set_level_prediction(False)
            ref.build(tp, eps=0.01, theta=theta)
            a2, p2 = ref.evaluate(tp, tm, p=4)
            torch.cuda.synchronize()
            assert i1 == ref.tree_info(), (precision, k)
            assert torch.equal(a1, a2) and torch.equal(p1, p2), (precision, k)
            ref.close()
        fused.close()


@pytest.mark.parametrize("kernel", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_forces_equals_build_then_evaluate(kernel, precision):
    """forces() runs the mass gather, P2M and M2M on the second stream beside
    the walk; the result equals build() followed by evaluate() bit for bit,
    on repeated calls and on a second system of another size."""
    torch, F = _torch(), _F()
    s1 = F.Solver(40000, p_max=5, leaf_size=24, kernel=kernel, precision=precision)
    s2 = F.Solver(40000, p_max=5, leaf_size=24, kernel=kernel, precision=precision)
    for k, (pos, _, m) in enumerate([W.plummer(40000, seed=61), W.plummer(40000, seed=61),
                                     W.uniform_sphere(25000, seed=62)]):
        tp = torch.from_numpy(np.ascontiguousarray(pos)).cuda()
        tm = torch.from_numpy(np.ascontiguousarray(m)).cuda()
        a1, p1 = s1.forces(tp, tm, eps=0.01, theta=0.45, p=5)
        s2.build(tp, eps=0.01, theta=0.45)
        a2, p2 = s2.evaluate(tp, tm, p=5)
        torch.cuda.synchronize()
        assert torch.equal(a1, a2) and torch.equal(p1, p2), k
        assert s1.tree_info() == s2.tree_info(), k
    s1.close()
    s2.close()
