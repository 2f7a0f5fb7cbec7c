"""Request server (continuous batching of independent HHS simulations).

* a request's result is bit-identical whether it is served alone or in a mix
  where requests arrive while others are resident and memory admission makes
  some wait;
* a served request equals the same system stepped with hhs_step at the
  server's top-level step (last step cut to end at t_end);
* admission never exceeds the arena or the slot count, and frees everything;
* cancellation of queued and resident requests; argument errors.
"""
import numpy as np
import pytest

from conftest import gpu_available
from paper_1712_10116_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

PRM = dict(W.PARAMS[4])
T_END = 0.3   # four top-level steps of 1/16 and a cut last one
T_ENDS = [0.3, 0.2, 0.3, 0.25, 0.15]   # per request in the mixes: they finish at different steps


def _requests():
    out = []
    for i, n in enumerate([900, 2500, 1300, 3100, 700]):
        gen = W.plummer if i % 2 == 0 else W.king
        kw = dict(a=3 * np.pi / 16) if i % 2 == 0 else dict(henon=True)
        out.append(gen(n, seed=7000 + i, **kw))
    return out


def _solver(max_n, precision):
    from paper_1712_10116_amd import fmm as F
    return F.Solver(max_n, p_max=PRM["p"], leaf_size=PRM["leaf_size"], kernel=PRM["kernel"],
                    precision=precision)


def _server(s, arena, slots, eta1=0.0):
    from paper_1712_10116_amd import fmm as F
    return F.Server(s, eps=PRM["eps"], theta=PRM["theta"], p=PRM["p"], eta=PRM["eta"],
                    max_levels=PRM["max_levels"], arena_bytes=arena, max_slots=slots, eta1=eta1)


def _drain(srv, got, limit=10000):
    for _ in range(limit):
        nr, nq = srv.step()
        for r in srv.poll():
            got[r["id"]] = r
        if nr == 0 and nq == 0:
            return
    raise AssertionError("server did not drain")


@pytest.mark.parametrize("precision", [0, 1])
def test_alone_equals_mix(precision):
    from paper_1712_10116_amd import fmm as F
    reqs = _requests()
    fp = [F.Server.footprint(m.size, PRM["max_levels"]) for _, _, m in reqs]
    s = _solver(4096, precision)
    # alone: one request at a time
    alone = []
    srv = _server(s, max(fp), 1)
    for k, (pos, vel, m) in enumerate(reqs):
        got = {}
        rid = srv.submit(pos, vel, m, T_ENDS[k])
        _drain(srv, got)
        alone.append(got[rid])
    srv.close()
    # mix: room for about two requests; three arrive first, two more after a step
    srv = _server(s, sorted(fp)[-1] + sorted(fp)[-2] + 4096, 3)
    got, ids = {}, []
    for k in range(3):
        ids.append(srv.submit(*reqs[k], T_ENDS[k]))
    nr, nq = srv.step()
    assert (nr, nq) == (3, 0)
    for k in range(3, 5):
        ids.append(srv.submit(*reqs[k], T_ENDS[k]))   # arrive while three are resident
    waited = False
    for _ in range(10000):
        nr, nq = srv.step()
        info = srv.info()
        assert nr <= 3 and info["arena_used"] <= info["arena_bytes"]
        waited = waited or nq > 0
        for r in srv.poll():
            got[r["id"]] = r
        if nr == 0 and nq == 0:
            break
    assert waited                    # the largest request had to wait for memory
    assert srv.info()["arena_used"] == 0
    for k, rid in enumerate(ids):
        a, b = alone[k], got[rid]
        assert np.array_equal(a["pos"], b["pos"]) and np.array_equal(a["vel"], b["vel"]), k
        for f in ("steps", "force_calls", "force_particles", "dt_top", "t_end"):
            assert a[f] == b[f], (k, f)
        assert b["t_submit"] <= b["t_admit"] <= b["t_done"]
    srv.close()
    s.close()


@pytest.mark.parametrize("eta1", [0.0, 0.0005])
def test_server_equals_hhs_step(eta1):
    """Also with the total-acceleration bound of Eq. (9) (eta1 > 0)."""
    import torch
    from paper_1712_10116_amd import fmm as F
    pos, vel, m = _requests()[1]
    s = _solver(4096, 0)
    srv = _server(s, F.Server.footprint(m.size, PRM["max_levels"]), 1, eta1)
    got = {}
    rid = srv.submit(pos, vel, m, T_END)
    _drain(srv, got)
    r = got[rid]
    srv.close()
    kw = dict(eps=PRM["eps"], theta=PRM["theta"], p=PRM["p"], eta=PRM["eta"],
              max_levels=PRM["max_levels"], eta1=eta1)
    h = F.HHS(s, torch.from_numpy(pos.copy()).cuda(), torch.from_numpy(vel.copy()).cuda(),
              torch.from_numpy(m).cuda(), **kw)
    h.init()
    amin = float(h.a_cur.min())
    dt = min(1.0 / 16, 2.0 ** np.floor(np.log2(np.sqrt(PRM["eta"] * PRM["eps"] / amin))))
    assert r["dt_top"] == dt
    t, steps, calls = 0.0, 0, 0
    while True:
        left = T_END - t
        last = dt >= left
        calls += h.step(left if last else dt)["force_calls"]
        t = h.t
        steps += 1
        if last:
            break
    torch.cuda.synchronize()
    assert steps == r["steps"] and calls == r["force_calls"] and t == r["t_end"]
    assert np.array_equal(h.pos.cpu().numpy(), r["pos"])
    assert np.array_equal(h.vel.cpu().numpy(), r["vel"])
    s.close()


def test_cancel_and_errors():
    from paper_1712_10116_amd import fmm as F
    reqs = _requests()
    fp = max(F.Server.footprint(m.size, PRM["max_levels"]) for _, _, m in reqs)
    s = _solver(4096, 1)
    srv = _server(s, fp, 1)
    ids = [srv.submit(pos, vel, m, T_END) for pos, vel, m in reqs[:3]]
    srv.step()                       # request 0 resident, 1 and 2 queued
    srv.cancel(ids[1])               # queued
    srv.cancel(ids[0])               # resident
    assert srv.info()["arena_used"] == 0
    got = {}
    _drain(srv, got)
    assert set(got) == {ids[2]}
    with pytest.raises(F.FMMError):
        srv.cancel(ids[0])
    big = W.plummer(5000, seed=1)
    with pytest.raises(F.FMMError) as e:
        srv.submit(*big, T_END)      # larger than max_n
    assert e.value.status == F.FMM_EINVAL
    srv.close()
    small = _server(s, F.Server.footprint(reqs[3][2].size, PRM["max_levels"]) - 4096, 1)
    with pytest.raises(F.FMMError) as e:
        small.submit(*reqs[3], T_END)  # footprint above the arena
    assert e.value.status == F.FMM_ENOMEM
    small.close()
    s.close()


def test_open_loop_driver():
    """The Poisson driver hands every request over and reports sane latencies."""
    from paper_1712_10116_amd import fmm as F
    from paper_1712_10116_amd import serving
    reqs = _requests()
    s = _solver(8192, 1)
    srv = _server(s, 64 << 20, 8)
    arr = serving.poisson_arrivals(len(reqs), rate=50.0, seed=3)
    res, span = serving.run(srv, reqs, 0.125, arrivals=arr)
    st = serving.summary(res, span)
    assert st["requests"] == len(reqs) and all(r is not None for r in res)
    assert all(r["latency"] > 0 and r["done"] >= r["arrival"] for r in res)
    assert st["p99_s"] >= st["p50_s"] > 0
    srv.close()
    s.close()


def test_many_residents_alone_equals_mix():
    """More residents than one batched integrator launch takes (16): 20 small
    requests arriving in three waves while others are part-way through their
    top-level steps end bit-identical to each served alone."""
    from paper_1712_10116_amd import fmm as F
    reqs = [(W.plummer if k % 2 else W.king)(200 + 23 * k, seed=7100 + k,
                                             **({} if k % 2 else dict(henon=True)))
            for k in range(20)]
    t_end = [0.125 if k % 3 else 0.1875 for k in range(20)]
    fp = sum(F.Server.footprint(m.size, PRM["max_levels"]) for _, _, m in reqs)
    s = _solver(8192, 1)
    alone = []
    srv = _server(s, fp, 1)
    for k, (pos, vel, m) in enumerate(reqs):
        got = {}
        rid = srv.submit(pos, vel, m, t_end[k])
        _drain(srv, got)
        alone.append(got[rid])
    srv.close()
    srv = _server(s, fp + (1 << 20), 20)
    got, ids = {}, []
    for wave in (range(0, 8), range(8, 15), range(15, 20)):
        for k in wave:
            ids.append(srv.submit(*reqs[k], t_end[k]))
        for _ in range(3):
            srv.step()
            for r in srv.poll():
                got[r["id"]] = r
    _drain(srv, got)
    assert len(got) == 20
    for k, rid in enumerate(ids):
        a, b = alone[k], got[rid]
        assert np.array_equal(a["pos"], b["pos"]) and np.array_equal(a["vel"], b["vel"]), k
        for f in ("steps", "force_calls", "force_particles", "dt_top", "t_end"):
            assert a[f] == b[f], (k, f)
    srv.close()
    s.close()
