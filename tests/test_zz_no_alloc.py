"""fmm_invariants_noalloc (no allocation, device output) against
fmm_invariants on the same arrays, bit for bit: two calls in a row, the
second on a smaller input, and a momentum-only call with NULL arrays."""
import numpy as np
import pytest

from conftest import gpu_available
from paper_1712_10116_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def test_noalloc_invariants_equal_allocating_entry():
    import torch
    from paper_1712_10116_amd import fmm as F
    pos, vel, m = W.plummer(30000, seed=1300)
    vel = vel + np.array([[0.2], [-0.1], [0.05]])
    s = F.Solver(30000, p_max=4, leaf_size=16, kernel=F.WENDLAND, precision=F.FP64)
    tp, tv, tm = (torch.from_numpy(x.copy()).cuda() for x in (pos, vel, m))
    a, pt = s.forces(tp, tm, eps=0.01, theta=0.5, p=4)
    out = torch.full((12,), float("nan"), dtype=torch.float64, device="cuda:0")
    for n in (30000, 7001):     # second call smaller: stale partials must not leak in
        args = [x[..., :n].contiguous() for x in (tp, tv, tm, a, pt)]
        ref = s.invariants(*args)
        F.invariants_noalloc(out, *args)
        got = out.cpu().numpy()
        want = np.concatenate([ref["F"], ref["P"], ref["L"], [ref["T"], ref["W"], ref["Fabs"]]])
        assert np.array_equal(got, want), (n, got - want)
    # NULL arrays: momentum of unit masses only
    F.invariants_noalloc(out, vel=tv)
    ref = s.invariants(vel=tv)
    got = out.cpu().numpy()
    assert np.array_equal(got[3:6], ref["P"]) and np.all(got[[0, 1, 2, 6, 7, 8, 10, 11]] == 0)
    # empty input: all zeros
    F.invariants_noalloc(out, vel=tv[:, :0].contiguous(), n=0)
    assert np.all(out.cpu().numpy() == 0)
    with pytest.raises(F.FMMError):
        F.invariants_noalloc(out, vel=tv, n=-1)
    s.close()
