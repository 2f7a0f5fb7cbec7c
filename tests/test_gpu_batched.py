"""Batched (forest) solves: several independent systems in one set of
launches.  Each system's results must be bit-identical to a solve of that
system alone (it has its own root box, keys and tree, and its cells never meet
another system's), and match the oracle (FP64 1e-12)."""
import numpy as np
import pytest

from conftest import gpu_available
from paper_1712_10116_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _systems():
    out = []
    for k, n in enumerate([1500, 0, 1, 4096, 700, 6000, 2]):
        if n == 0:
            pos = np.zeros((3, 5))
            m = np.ones(5)
            act = np.zeros(0, dtype=np.int32)
        else:
            gen = W.plummer if k % 2 else W.uniform_sphere
            pos, _, m = gen(max(n, 3), seed=900 + k)
            pos = pos[:, :n] + 10.0 * k   # far apart and at different offsets
            m = m[:n]
            act = None
            if k == 3:
                act = np.random.default_rng(k).permutation(n)[: n // 2].astype(np.int32)
        out.append((pos, m, act))
    return out


@pytest.mark.parametrize("precision,kernel", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_batched_equals_solo(oracle, precision, kernel):
    import torch
    from paper_1712_10116_amd import fmm as F
    systems = _systems()
    total = sum(len(m) if a is None else len(a) for _, m, a in systems)
    s = F.Solver(total, p_max=5, leaf_size=16, kernel=kernel, precision=precision)
    dev = [dict(pos=torch.from_numpy(np.ascontiguousarray(p)).cuda(),
                mass=torch.from_numpy(np.ascontiguousarray(m)).cuda(),
                active=None if a is None else torch.from_numpy(a).cuda()) for p, m, a in systems]
    outs = s.forces_batched(dev, eps=0.01, theta=0.5, p=5)
    info = s.tree_info()
    torch.cuda.synchronize()
    batched = [(a.cpu().numpy(), p.cpu().numpy()) for a, p in outs]
    nodes = 0
    for k, d in enumerate(dev):
        a, pt = s.forces(d["pos"], d["mass"], d["active"], eps=0.01, theta=0.5, p=5)
        nodes += s.tree_info()["nodes"]
        torch.cuda.synchronize()
        assert np.array_equal(a.cpu().numpy(), batched[k][0]), k
        assert np.array_equal(pt.cpu().numpy(), batched[k][1]), k
        pos, m, act = systems[k]
        if precision == 0 and (len(m) if act is None else len(act)) > 1:
            ra, rp = oracle.fmm(pos, m, act, p=5, theta=0.5, eps=0.01, leaf_size=16, kernel=kernel)
            mag = np.sqrt((ra ** 2).sum(axis=0))
            floor = 1e-6 * np.sqrt((mag ** 2).mean())
            e = np.sqrt(((batched[k][0] - ra) ** 2).sum(axis=0)) / np.maximum(mag, floor)
            assert e.max() < 1e-12
    assert info["nodes"] == nodes
    s.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_small_batch_paths_identical(precision):
    """A batch small enough for the single-workgroup build (several requests,
    so the sort also orders by request) equals the multi-workgroup build bit
    for bit, and each system equals its solo solve."""
    import torch
    from paper_1712_10116_amd import fmm as F
    sizes = [1500, 0, 1, 2000, 700, 3000, 2]
    dev = []
    for (p, m, _), n in zip(_systems(), sizes):
        if n == 0:  # an empty system: active set of size zero
            dev.append(dict(pos=torch.from_numpy(np.ascontiguousarray(p)).cuda(),
                            mass=torch.from_numpy(np.ascontiguousarray(m)).cuda(),
                            active=torch.zeros(0, dtype=torch.int32, device="cuda")))
            continue
        dev.append(dict(pos=torch.from_numpy(np.ascontiguousarray(p[:, :n])).cuda(),
                        mass=torch.from_numpy(np.ascontiguousarray(m[:n])).cuda(), active=None))
    total = sum(d["mass"].numel() if d["active"] is None else 0 for d in dev)
    assert total <= 8192
    res = []
    for small in (True, False):
        s = F.Solver(total, p_max=4, leaf_size=16, kernel=0, precision=precision)
        s.set_small_path(2 if small else False)
        outs = s.forces_batched(dev, eps=0.01, theta=0.5, p=4)
        torch.cuda.synchronize()
        res.append([(a.cpu().numpy(), p.cpu().numpy()) for a, p in outs])
        if small:
            for k, d in enumerate(dev):
                a, pt = s.forces(d["pos"], d["mass"], d["active"], eps=0.01, theta=0.5, p=4)
                torch.cuda.synchronize()
                assert np.array_equal(a.cpu().numpy(), res[0][k][0]), k
        s.close()
    for (a1, p1), (a2, p2) in zip(*res):
        assert np.array_equal(a1, a2) and np.array_equal(p1, p2)
