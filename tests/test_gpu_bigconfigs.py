"""GPU parity at the full sizes of the disk-galaxy and clustered-zoom
workloads, in the launch configuration the benchmark's per-workload leg times
them (their own p and theta, leaf 64, solved by fmm_forces):

* disk galaxy, N = 2^22 (exponential disk, Hernquist bulge, NFW halo with 8x
  heavier particles), Wendland eps = 0.02, p = 6, theta = 0.4;
* clustered zoom, N = 2^24 (2000 NFW halos plus a uniform background of 8x
  heavier particles), Wendland eps = 0.001, p = 6, theta = 0.4;

tree, permutation and both interaction lists bit-exact against the oracle;
FP64 forces and potentials within 1e-12 of the oracle on seeded sinks
(evaluated sink by sink), mixed precision within 2e-6 rms on the same sinks.
"""
import numpy as np
import pytest

from conftest import gpu_available
from paper_1712_10116_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.slow,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

CASES = {"disk_2^22": (2, 64, 256), "zoom_2^24": (3, 64, 64)}


@pytest.fixture(scope="module", params=list(CASES))
def big(request, oracle):
    c, leaf, ns = CASES[request.param]
    pos, _, m = W.config(c)
    prm = dict(W.PARAMS[c])
    t = oracle.Tree(pos, p=prm["p"], theta=prm["theta"], eps=prm["eps"], leaf_size=leaf,
                    kernel=prm["kernel"])
    sinks = np.sort(np.random.default_rng(700 + c).choice(m.size, ns, replace=False))
    ra, rp = t.evaluate_sinks(m, sinks)
    yield c, leaf, prm, pos, m, t, sinks, ra, rp
    del t


def _solve(pos, m, prm, leaf, precision, export):
    import torch
    from paper_1712_10116_amd import fmm as F
    s = F.Solver(m.size, p_max=prm["p"], leaf_size=leaf, kernel=prm["kernel"],
                 precision=precision)
    tp, tm = torch.from_numpy(pos).cuda(), torch.from_numpy(m).cuda()
    a, pt = s.forces(tp, tm, eps=prm["eps"], theta=prm["theta"], p=prm["p"])
    ex = s.export_tree() if export else None
    out = a.cpu().numpy(), pt.cpu().numpy(), ex
    s.close()
    del tp, tm, a, pt
    torch.cuda.empty_cache()
    return out


def test_big_tree_and_lists_bit_exact(big):
    c, leaf, prm, pos, m, t, *_ = big
    _, _, ex = _solve(pos, m, prm, leaf, 1, True)
    ref = t.export()
    for k in ("perm", "level", "prefix", "begin", "end", "is_leaf", "centre", "half", "box",
              "m2l", "p2p"):
        np.testing.assert_array_equal(ex[k], ref[k], err_msg=k)


@pytest.mark.parametrize("precision", [0, 1])
def test_big_forces(big, precision):
    c, leaf, prm, pos, m, t, sinks, ra, rp = big
    a, pt, _ = _solve(pos, m, prm, leaf, precision, False)
    mag = np.sqrt((ra * ra).sum(axis=0))
    e = np.sqrt(((a[:, sinks] - ra) ** 2).sum(axis=0)) / mag
    ep = np.abs(pt[sinks] - rp) / np.abs(rp)
    if precision == 0:
        assert e.max() < 1e-12 and ep.max() < 1e-12, (e.max(), ep.max())
    else:
        assert np.sqrt((e * e).mean()) < 2e-6 and np.sqrt((ep * ep).mean()) < 2e-6, (
            np.sqrt((e * e).mean()), np.sqrt((ep * ep).mean()))
