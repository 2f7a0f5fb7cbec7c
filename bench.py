#!/usr/bin/env python
"""FMM force-solve benchmark on one MI355X.

Workload: cold collapse -- 1,048,576 equal-mass particles uniform in the unit
sphere (G = M = R = 1), Wendland C2 softening eps = 0.005.  One step = one
complete force solve of all particles (root box, Morton keys and sort, tree,
symmetric dual walk, P2M/M2M, M2L, P2P, L2L/L2P) through the C ABI, inputs
resident in HBM.

The leaf size, opening angle and order are picked first by the autotuner (the
fastest mixed-precision solve whose rms force error over all particles, against
a high-accuracy FP64 solve, is within the target); the plain FP64 path runs at
the same parameters, so both have the same truncation error.  The workload's
own parameters (p 4, theta 0.5, leaf 16) are timed beside them.

Prints one JSON line: particles/s of the mixed-precision path (the headline),
the FP64 path beside it, force errors (all particles against the reference
solve; a seeded sample of sinks against FP64 direct summation by the CPU
oracle), momentum balance, per-phase HIP-event times, the roofline of the
dominant kernel, the CPU oracle timed on a bounded sample, one HHS top-level
step and the serving ensemble.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector (published)
PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector (published)
METRIC = "FMM force particles/s at 1e-3 force err (mixed vs FP64); ensemble p99 latency"


def progress(msg):
    """A progress line on stderr (stdout carries only the result line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def coeffs(p):
    return (p + 1) * (p + 2) * (p + 3) // 6


def m2l_flops_per_pair(p):
    # per unordered cell pair: both contractions (2 x 2 flops per term,
    # C(p+6,6) terms) plus one derivative tensor, about 2 C(p+3,3) (p+1) flops
    from math import comb
    return 4 * comb(p + 6, 6) + 2 * coeffs(p) * (p + 1)


P2P_FLOPS_PER_PAIR = 30.0  # per unordered particle pair (rsqrt counted as 1)


def recorded_traffic(kernel, prm):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None if it was taken for other parameters or the kernel sources changed since."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "hbm_traffic_cold_collapse_1M.md")
    if not os.path.exists(path):
        return None
    csrc = os.path.join(ROOT, "paper_1712_10116_amd", "csrc")
    sha = hashlib.sha256(open(os.path.join(csrc, "eval.hip"), "rb").read() +
                         open(os.path.join(csrc, "expansion.h"), "rb").read()).hexdigest()
    for m in re.finditer(r"traffic_bytes_per_launch: (.*)", open(path).read()):
        kv = dict(x.split("=", 1) for x in m.group(1).split())
        same = (kv.get("p") == str(prm["p"]) and kv.get("theta") == str(prm["theta"]) and
                kv.get("leaf") == str(prm["leaf_size"]))
        if kv.get("source_sha256") == sha and same and kernel in kv:
            return int(kv[kernel])
    return None


def force_error(acc, ref):
    mag = np.sqrt((ref * ref).sum(axis=0))
    floor = 1e-6 * np.sqrt((mag * mag).mean())
    e = np.sqrt(((acc - ref) ** 2).sum(axis=0)) / np.maximum(mag, floor)
    return float(np.sqrt((e * e).mean())), float(np.percentile(e, 99))


def time_solver(F, torch, s, tp, tm, acc, pot, prm, steps, warmup, profile):
    """Seconds per solve over `steps` timed solves.  With `profile`: HIP events
    around the M2L and P2P kernels inside the timed region (their launch
    durations, for the roofline), and the per-phase event times of a further
    `steps` solves outside it (events between every phase lengthen a solve).
    Returns (seconds, phases summed over the profiled solves, kernel times
    summed over the timed solves)."""
    for _ in range(warmup):
        s.forces(tp, tm, eps=prm["eps"], theta=prm["theta"], p=prm["p"], acc=acc, pot=pot)
    torch.cuda.synchronize()
    if profile:
        s.profile(True, kernels_only=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s.forces(tp, tm, eps=prm["eps"], theta=prm["theta"], p=prm["p"], acc=acc, pot=pot)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phases = kern = None
    if profile:
        kern = s.profile_read()
        s.profile(True)
        for _ in range(steps):
            s.forces(tp, tm, eps=prm["eps"], theta=prm["theta"], p=prm["p"], acc=acc, pot=pot)
        torch.cuda.synchronize()
        phases = s.profile_read()
        s.profile(False)
    return (t1 - t0) / steps, phases, kern


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_leg(args, n, pos, mass, res, prm, line):
    """CPU side: FP64 direct summation (oracle) on a seeded sample of sinks as
    the force-error reference of every GPU result, and the oracle FMM timed
    twice: the whole workload on all host cores (its OpenMP evaluation, equal
    to the single-threaded one bit for bit), and the single-threaded oracle on
    a bounded sample of the same recipe."""
    from oracle import oracle as O
    from paper_1712_10116_amd import workloads as W
    rng = np.random.default_rng(2024)
    sinks = np.sort(rng.choice(n, size=min(args.sample, n), replace=False))
    ref, _ = O.direct(pos, mass, O.WENDLAND, 0.005, sinks=sinks)
    for name, r in res.items():
        e = force_error(r["acc"][:, sinks], ref)
        line["force_err"]["vs_direct_sample"][name] = {"rms": e[0], "p99": e[1]}
    line["force_err"]["vs_direct_sample"]["sinks"] = int(len(sinks))
    kw = dict(p=prm["p"], theta=prm["theta"], eps=0.005, leaf_size=prm["leaf_size"],
              kernel=O.WENDLAND)
    # all cores, the whole workload: tree build + evaluation, best of up to
    # three runs (fewer when one takes more than 15 s)
    threads = O.threads()
    best = None
    for _ in range(3):
        t0 = time.perf_counter()
        t = O.Tree(pos, **kw)
        t.evaluate_parallel(mass)
        dt = time.perf_counter() - t0
        del t
        best = dt if best is None else min(best, dt)
        if dt > 15.0:
            break
    # one thread: the plain oracle on a sample of about 10-30 s of work,
    # doubled while the solve takes under 10 s
    ns = min(args.cpu_sample, n)
    while True:
        spos, _, smass = W.uniform_sphere(ns, seed=1001)
        t0 = time.perf_counter()
        O.fmm(spos, smass, **kw)
        t1 = time.perf_counter()
        if t1 - t0 >= 10.0 or ns >= n or 2.2 * (t1 - t0) > 40.0:
            break
        ns = min(n, 2 * ns)
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    line["cpu_baseline"] = {
        "value": round(n / best, 1), "unit": "particles/s", "cores": threads, "kind": "oracle",
        "sample": f"the whole workload ({n} particles, p={prm['p']}, theta={prm['theta']}, leaf "
                  f"{prm['leaf_size']}): one oracle FMM force solve (FP64, tree build and "
                  f"evaluation) with its evaluation on {threads} OpenMP threads, best of the "
                  f"runs, {best:.2f} s",
        "cpu_model": cpu_model(), "host_cpus": os.cpu_count(), "cpus_available": affinity,
        "single_thread": {"value": round(ns / (t1 - t0), 1), "unit": "particles/s",
                          "sample": f"the single-threaded oracle on a {ns}-particle uniform "
                                    f"sphere of the same recipe, {t1 - t0:.1f} s"}}


def chin_leg(args, F, torch, line):
    """The fourth-order integrator of Sec. 4.1 (chin_step) against the KDK
    leapfrog at equal force evaluations: a Plummer sphere of 65,536 particles
    (Plummer softening, FP64, p 6, leaf 64; theta 0.4, and theta 1e-6 where
    every pair is summed directly) advanced to t = 1,
    Chin with h = 1/16 (16 steps, 1 + 3 x 16 evaluations) against KDK with h =
    1/48 (48 steps, the closing kick's acceleration reused by the next
    opening kick: 1 + 48 evaluations); the energy is measured after every
    Chin step and every third KDK step (same times) by an FP64 direct sum,
    and the largest relative error of each run is reported.  The KDK kicks
    and drifts are torch additions around the library's solves."""
    from paper_1712_10116_amd import workloads as W
    dev = torch.device("cuda:0")
    n, t_end, hc = 65536, 1.0, 1.0 / 16
    pos, vel, m = W.plummer(n, seed=1500)
    tm = torch.from_numpy(m).to(dev)
    out = {"n": n, "t_end": t_end, "h_chin": hc, "h_kdk": hc / 3, "precision": "fp64",
           "p": 6, "leaf_size": 64, "kernel": "plummer", "runs": []}
    # the FMM at theta 0.4, and every pair summed directly (theta 1e-6), where
    # the solver's truncation error no longer adds to the integration error
    for eps, theta in ((0.1, 0.4), (0.1, 1e-6), (0.3, 1e-6)):
        kw = dict(eps=eps, theta=theta, p=6)
        s = F.Solver(n, p_max=6, leaf_size=64, kernel=F.PLUMMER, precision=F.FP64)
        e = F.Solver(n, p_max=4, leaf_size=64, kernel=F.PLUMMER, precision=F.FP64)

        def energy(tp, tv):
            _, pot = e.forces(tp, tm, eps=eps, theta=1e-6, p=4)
            inv = e.invariants(vel=tv, mass=tm, pot=pot)
            return inv["T"] + inv["W"]

        steps = int(round(t_end / hc))
        tp = torch.from_numpy(pos.copy()).to(dev)
        tv = torch.from_numpy(vel.copy()).to(dev)
        E0 = energy(tp, tv)
        c = F.Chin(s, tp, tv, tm, **kw)
        c.init()
        dc, sec_c = [], 0.0
        for _ in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c.step(hc)
            torch.cuda.synchronize()
            sec_c += time.perf_counter() - t0
            dc.append(abs(energy(tp, tv) / E0 - 1))
        tp = torch.from_numpy(pos.copy()).to(dev)
        tv = torch.from_numpy(vel.copy()).to(dev)
        a, _ = s.forces(tp, tm, **kw)
        h = hc / 3
        dk, sec_k = [], 0.0
        for k in range(3 * steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tv.add_(a, alpha=h / 2)
            tp.add_(tv, alpha=h)
            a, _ = s.forces(tp, tm, **kw)
            tv.add_(a, alpha=h / 2)
            torch.cuda.synchronize()
            sec_k += time.perf_counter() - t0
            if k % 3 == 2:
                dk.append(abs(energy(tp, tv) / E0 - 1))
        s.close()
        e.close()
        out["runs"].append({"eps": eps, "theta": theta, "evaluations": 1 + 3 * steps,
                            "chin": {"max_energy_err": max(dc), "seconds": round(sec_c, 4)},
                            "kdk": {"max_energy_err": max(dk), "seconds": round(sec_k, 4)},
                            "kdk_over_chin": round(max(dk) / max(max(dc), 1e-300), 2)})
    line["chin"] = out


def ensemble_leg(args, F, torch, line):
    """Serving: an ensemble of independent HHS simulations (Plummer / King
    W0 = 6 in Henon units, N log-uniform in [1024, 262144]) each advanced to
    t = t_end through the request server.  First a closed loop (all requests
    at once) measures the saturation rate; then Poisson arrivals at a fraction
    of it give the p50/p99 latency; a few requests served alone give the
    latency without contention."""
    from paper_1712_10116_amd import serving
    from paper_1712_10116_amd import workloads as W
    from paper_1712_10116_amd import autotune
    prm = dict(W.PARAMS[4])
    K = args.ensemble
    reqs = [W.ensemble_request(i) for i in range(K)]
    ntot = sum(r[2].size for r in reqs)
    # leaf size by the autotuner on the serving workload itself: a short closed
    # loop (the first 64 requests, one top-level step each) per candidate; with
    # 16 the loop is too lightly loaded to rank leaf 32 against 64 as the full
    # stream does
    probe = reqs[:64]

    def probe_run(leaf):
        sv = F.Solver(args.ensemble_max_n, p_max=prm["p"], leaf_size=leaf, kernel=prm["kernel"],
                      precision=F.MIXED)
        srv = F.Server(sv, eps=prm["eps"], theta=prm["theta"], p=prm["p"], eta=prm["eta"],
                       max_levels=prm["max_levels"], arena_bytes=args.ensemble_arena_gib << 30,
                       max_slots=args.ensemble_slots)
        _, span = serving.run(srv, probe, 1.0 / 16)
        srv.close()
        sv.close()
        return span

    tl = autotune.fastest((16, 32, 64, 96, 128), probe_run)
    prm["leaf_size"] = tl["best"]
    s = F.Solver(args.ensemble_max_n, p_max=prm["p"], leaf_size=prm["leaf_size"],
                 kernel=prm["kernel"], precision=F.MIXED)

    def server():
        return F.Server(s, eps=prm["eps"], theta=prm["theta"], p=prm["p"], eta=prm["eta"],
                        max_levels=prm["max_levels"], arena_bytes=args.ensemble_arena_gib << 30,
                        max_slots=args.ensemble_slots)

    srv = server()
    serving.run(srv, [W.ensemble_request(1000)], args.ensemble_t_end)  # warm-up, untimed
    progress("  closed loop")
    res, span = serving.run(srv, reqs, args.ensemble_t_end,
                            log=lambda m: progress("    " + m) if K > 64 else None)
    closed = serving.summary(res, span)
    rate = args.ensemble_load * closed["requests_per_s"]
    arr = serving.poisson_arrivals(K, rate, seed=5999)
    progress(f"  Poisson arrivals at {rate:.3f} per s")
    res, span = serving.run(srv, reqs, args.ensemble_t_end, arrivals=arr,
                            log=lambda m: progress("    " + m) if K > 64 else None)
    opened = serving.summary(res, span)
    # latency alone: the smallest, the median-size and the largest request
    sizes = np.array([r[2].size for r in reqs])
    pick = sorted({int(np.argmin(sizes)), int(np.argsort(sizes)[K // 2]), int(np.argmax(sizes))})
    solo = {}
    for k in pick:
        rr, sp = serving.run(srv, [reqs[k]], args.ensemble_t_end)
        solo[int(sizes[k])] = round(rr[0]["latency"], 4)
    srv.close()
    s.close()
    rnd = lambda d: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}
    line["ensemble"] = {
        "requests": K, "particles": int(ntot), "t_end": args.ensemble_t_end,
        "precision": "mixed", "p": prm["p"], "theta": prm["theta"], "eps": prm["eps"],
        "leaf_size": prm["leaf_size"],
        "leaf_tuning_s": {str(r["candidate"]): round(r["seconds"], 4) for r in tl["table"]},
        "arena_gib": args.ensemble_arena_gib, "max_slots": args.ensemble_slots,
        "closed_loop": rnd(closed),
        "poisson": dict(rnd(opened), rate_per_s=round(rate, 4), load=args.ensemble_load),
        "p50_latency_s": round(opened["p50_s"], 4), "p99_latency_s": round(opened["p99_s"], 4),
        "solo_latency_s_by_n": solo,
    }


def configs_leg(args, F, torch, line):
    """Every named workload at its own p and theta (leaf size by the
    autotuner): one timed solve, force error over all particles against the
    high-accuracy FP64 solve and on seeded sinks against FP64 direct summation
    (CPU oracle), momentum balance; HHS runs on the Plummer sphere (8 steps,
    FP64) and the cold collapse (to two free-fall times, mixed) with the drift
    of total momentum and angular momentum."""
    from paper_1712_10116_amd import autotune
    from paper_1712_10116_amd import workloads as W
    names = {0: "plummer_4096", 1: "cold_collapse_2^20", 2: "disk_galaxy_2^22",
             3: "clustered_zoom_2^24"}
    precision = {0: F.FP64, 1: F.MIXED, 2: F.MIXED, 3: F.MIXED}
    sinks_n = {0: 4096, 1: 1024, 2: 512, 3: 256}
    dev = torch.device("cuda:0")
    out = {}
    for c in args.configs:
        progress(f"config {names[c]}")
        prm = W.PARAMS[c]
        pos, vel, m = W.config(c)
        n = m.size
        tp = torch.from_numpy(pos).to(dev)
        tm = torch.from_numpy(m).to(dev)
        tr = autotune.tune(tp, tm, eps=prm["eps"], kernel=prm["kernel"], precision=precision[c],
                           target=None, leaf_sizes=(16, 32, 64, 96), orders=(prm["p"],),
                           thetas=(prm["theta"],), reps=3)
        leaf = tr["best"]["leaf_size"]
        s = F.Solver(n, p_max=prm["p"], leaf_size=leaf, kernel=prm["kernel"],
                     precision=precision[c])
        acc = torch.empty((3, n), dtype=torch.float64, device=dev)
        pot = torch.empty((n,), dtype=torch.float64, device=dev)
        pr = dict(p=prm["p"], theta=prm["theta"], eps=prm["eps"])
        sec, _, _ = time_solver(F, torch, s, tp, tm, acc, pot, pr, 5, 1, profile=False)
        inv = s.invariants(mass=tm, acc=acc)
        a = acc.cpu().numpy()
        s.close()
        sec64 = None
        if precision[c] == F.MIXED:  # the plain FP64 path at the same parameters
            s = F.Solver(n, p_max=prm["p"], leaf_size=leaf, kernel=prm["kernel"],
                         precision=F.FP64)
            sec64, _, _ = time_solver(F, torch, s, tp, tm, acc, pot, pr, 5, 1, profile=False)
            s.close()
        rp = autotune.REFERENCE
        r = F.Solver(n, p_max=rp["p"], leaf_size=rp["leaf_size"], kernel=prm["kernel"],
                     precision=F.FP64)
        a_ref, _ = r.forces(tp, tm, eps=prm["eps"], theta=rp["theta"], p=rp["p"])
        a_ref = a_ref.cpu().numpy()
        r.close()
        e_all = force_error(a, a_ref)
        row = {"n": n, "p": prm["p"], "theta": prm["theta"], "eps": prm["eps"], "leaf_size": leaf,
               "kernel": "plummer" if prm["kernel"] == F.PLUMMER else "wendland_c2",
               "precision": "fp64" if precision[c] == F.FP64 else "mixed",
               "ms_per_solve": round(sec * 1e3, 4), "particles_per_s": round(n / sec, 1),
               "force_err_vs_reference_all": {"rms": e_all[0], "p99": e_all[1]},
               "momentum_rel": float(np.abs(inv["F"]).max() / inv["Fabs"])}
        if sec64 is not None:
            row["fp64"] = {"ms_per_solve": round(sec64 * 1e3, 4),
                           "particles_per_s": round(n / sec64, 1)}
        if not args.no_cpu_baseline:
            from oracle import oracle as O
            rng = np.random.default_rng(3000 + c)
            sk = np.sort(rng.choice(n, size=min(sinks_n[c], n), replace=False))
            d, _ = O.direct(pos, m, O.PLUMMER if prm["kernel"] == F.PLUMMER else O.WENDLAND,
                            prm["eps"], sinks=sk)
            e = force_error(a[:, sk], d)
            row["force_err_vs_direct_sample"] = {"rms": e[0], "p99": e[1], "sinks": int(len(sk))}
        # HHS: 8 steps of the Plummer sphere, the cold collapse to t_end, one
        # top-level step of the disk (14 rungs) and of the zoom (16 rungs)
        steps, t_end = {0: (8, None), 1: (None, args.collapse_t_end), 2: (1, None),
                        3: (1, None)}.get(c, (0, None))
        if steps or t_end:
            s = F.Solver(n, p_max=prm["p"], leaf_size=leaf, kernel=prm["kernel"],
                         precision=precision[c])
            tv = torch.from_numpy(vel).to(dev)
            tpp = tp.clone()
            h = F.HHS(s, tpp, tv, tm, eps=prm["eps"], theta=prm["theta"], p=prm["p"],
                      eta=prm["eta"], max_levels=prm["max_levels"])
            h.init()
            dtmax = float(np.sqrt(prm["eta"] * prm["eps"] /
                                  max(float(h.a_cur[h.a_cur > 0].min()), 1e-30)))
            dt_top = min(2.0 ** np.floor(np.log2(dtmax)), 2.0 ** -4)
            i0 = s.invariants(pos=tpp, vel=tv, mass=tm)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            k = 0
            calls = parts = 0
            while (steps and k < steps) or (t_end and h.t < t_end - 1e-12):
                dt = dt_top if not t_end else min(dt_top, t_end - h.t)
                st = h.step(dt)
                calls += st["force_calls"]
                parts += st["force_particles"]
                k += 1
                progress(f"  {names[c]} HHS step {k}: t = {h.t:.4f}, {st['force_calls']} calls")
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            i1 = s.invariants(pos=tpp, vel=tv, mass=tm)
            pscale = float(np.sum(m * np.sqrt((vel * vel).sum(axis=0)))) or 1.0
            lscale = float(np.sum(m * np.sqrt((pos * pos).sum(axis=0)) *
                                  np.sqrt((vel * vel).sum(axis=0)))) or 1.0
            row["hhs"] = {"steps": k, "t": h.t, "dt_top": dt_top, "seconds": round(wall, 3),
                          "force_calls": calls, "particles_per_s": round(parts / wall, 1),
                          "momentum_drift": float(np.abs(i1["P"] - i0["P"]).max()),
                          "momentum_scale": pscale if c == 0 else None,
                          "angular_momentum_drift": float(np.abs(i1["L"] - i0["L"]).max()),
                          "kinetic_energy": [i0["T"], i1["T"]],
                          "rung_histogram": torch.bincount(h.rung.long()).cpu().numpy().tolist()}
            if c != 0:  # a cold start has no momentum scale of its own: use m |a| dt
                row["hhs"]["momentum_scale"] = float(inv["Fabs"]) * h.t
            s.close()
        out[names[c]] = row
        del tp, tm, acc, pot
        torch.cuda.empty_cache()
    line["configs"] = out


def graph_ab_leg(args):
    """A/B of HIP-graph replay against direct launches for one evaluation on a
    fixed tree (the pattern of the two kicks of a KDK half, which share a
    tree): seconds per evaluation each way and the capture + instantiation
    cost, for a few system sizes (mixed, Wendland, p 4, leaf 16).  Every
    replay's result is compared with the direct one.  Prints one JSON line."""
    import torch
    import paper_1712_10116_amd.fmm as F
    from paper_1712_10116_amd import workloads as W
    dev = torch.device("cuda:0")
    out = {}
    for n in (2048, 12526, 65536):
        pos, _, m = W.plummer(n, seed=7)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            s = F.Solver(n, p_max=4, leaf_size=16, kernel=F.WENDLAND, precision=F.MIXED,
                         stream=stream)
            tp, tm = torch.from_numpy(pos).to(dev), torch.from_numpy(m).to(dev)
            acc = torch.empty((3, n), dtype=torch.float64, device=dev)
            pot = torch.empty(n, dtype=torch.float64, device=dev)
            s.build(tp, eps=0.01, theta=0.5)
            s.evaluate(tp, tm, p=4, acc=acc, pot=pot)
            torch.cuda.synchronize()
            ref = acc.clone()
            reps = args.graph_ab
            t0 = time.perf_counter()
            for _ in range(reps):
                s.evaluate(tp, tm, p=4, acc=acc, pot=pot)
            torch.cuda.synchronize()
            direct = (time.perf_counter() - t0) / reps
            g = torch.cuda.CUDAGraph()
            t0 = time.perf_counter()
            with torch.cuda.graph(g, stream=stream):
                s.evaluate(tp, tm, p=4, acc=acc, pot=pot)
            torch.cuda.synchronize()
            cap = time.perf_counter() - t0
            same = True
            for _ in range(3):   # replays between eager work, each checked
                acc.zero_()
                g.replay()
                torch.cuda.synchronize()
                same = same and bool(torch.equal(acc, ref))
            t0 = time.perf_counter()
            for _ in range(reps):
                g.replay()
            torch.cuda.synchronize()
            rep = (time.perf_counter() - t0) / reps
            same = same and bool(torch.equal(acc, ref))
            info = s.tree_info()
            out[str(n)] = {"direct_us": round(direct * 1e6, 1), "replay_us": round(rep * 1e6, 1),
                           "capture_instantiate_us": round(cap * 1e6, 1), "replays_equal": same,
                           "nodes": info["nodes"], "depth": info["depth"]}
            del g
            s.close()
    print(json.dumps({"graph_ab": out}))


def collapse_run_leg(args):
    """The cold collapse (uniform sphere at rest, Wendland eps = 0.005, p 4,
    theta 0.5, HHS with 10 rungs) integrated to t = collapse_t_end with N =
    collapse_run particles, in mixed precision and in FP64: total momentum and
    angular momentum drift, kinetic energy, force calls; prints one JSON line."""
    import torch
    import paper_1712_10116_amd.fmm as F
    from paper_1712_10116_amd import workloads as W
    prm = W.PARAMS[1]
    n = args.collapse_run
    pos, vel, m = W.uniform_sphere(n, seed=1001)
    out = {"n": n, "t_end": args.collapse_t_end, "p": prm["p"], "theta": prm["theta"],
           "eps": prm["eps"], "leaf_size": args.leaf}
    for name, prec in (("mixed", F.MIXED), ("fp64", F.FP64)):
        s = F.Solver(n, p_max=prm["p"], leaf_size=args.leaf, kernel=prm["kernel"], precision=prec)
        tp = torch.from_numpy(pos.copy()).cuda()
        tv = torch.from_numpy(vel.copy()).cuda()
        tm = torch.from_numpy(m).cuda()
        h = F.HHS(s, tp, tv, tm, eps=prm["eps"], theta=prm["theta"], p=prm["p"], eta=prm["eta"],
                  max_levels=prm["max_levels"])
        h.init()
        dtmax = float(np.sqrt(prm["eta"] * prm["eps"] /
                              max(float(h.a_cur[h.a_cur > 0].min()), 1e-30)))
        dt_top = min(2.0 ** np.floor(np.log2(dtmax)), 2.0 ** -4)
        fabs = s.invariants(mass=tm, acc=s.forces(tp, tm, eps=prm["eps"], theta=prm["theta"],
                                                  p=prm["p"])[0])["Fabs"]
        t0 = time.perf_counter()
        k = calls = 0
        while h.t < args.collapse_t_end - 1e-12:
            st = h.step(min(dt_top, args.collapse_t_end - h.t))
            calls += st["force_calls"]
            k += 1
            progress(f"{name} collapse step {k}: t = {h.t:.4f}, {st['force_calls']} calls")
        torch.cuda.synchronize()
        inv = s.invariants(pos=tp, vel=tv, mass=tm)
        out[name] = {"steps": k, "dt_top": dt_top, "seconds": round(time.perf_counter() - t0, 2),
                     "force_calls": calls, "momentum": inv["P"].tolist(),
                     "momentum_rel": float(np.abs(inv["P"]).max() / (fabs * h.t)),
                     "angular_momentum": inv["L"].tolist(), "kinetic_energy": float(inv["T"])}
        s.close()
    print(json.dumps(out))


def hhs_request_leg(args):
    """Top-level HHS steps (dt 1/16) of one ensemble request, after one
    untimed step; prints one JSON line."""
    import torch
    import paper_1712_10116_amd.fmm as F
    from paper_1712_10116_amd import workloads as W
    prm = dict(W.PARAMS[4])
    if args.hhs_leaf:
        prm["leaf_size"] = args.hhs_leaf
    pos, vel, m = W.ensemble_request(args.hhs_request)
    s = F.Solver(m.size, p_max=prm["p"], leaf_size=prm["leaf_size"], kernel=prm["kernel"],
                 precision=F.MIXED)
    s.set_small_path(args.hhs_small_path)
    s.set_level_prediction(args.hhs_predict)
    h = F.HHS(s, torch.from_numpy(pos).cuda(), torch.from_numpy(vel).cuda(),
              torch.from_numpy(m).cuda(), eps=prm["eps"], theta=prm["theta"], p=prm["p"],
              eta=prm["eta"], max_levels=prm["max_levels"])
    h.init()
    h.step(1.0 / 16)
    torch.cuda.synchronize()
    steps = []
    for _ in range(args.hhs_steps):
        t0 = time.perf_counter()
        st = h.step(1.0 / 16)
        torch.cuda.synchronize()
        steps.append(dict(ms=round((time.perf_counter() - t0) * 1e3, 3), **st))
    rungs = torch.bincount(h.rung.long()).cpu().numpy().tolist()
    print(json.dumps({"request": args.hhs_request, "n": int(m.size), "leaf_size": prm["leaf_size"],
                      "small_path": args.hhs_small_path, "level_prediction": args.hhs_predict,
                      "rung_histogram": rungs, "steps": steps}))
    s.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--target", type=float, default=1e-3, help="rms force error to reach")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner and use --p/--theta/--leaf")
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--p", type=int, default=6)
    ap.add_argument("--leaf", type=int, default=64)
    ap.add_argument("--sample", type=int, default=4096, help="sinks checked against direct sum")
    ap.add_argument("--cpu-sample", type=int, default=262144, help="particles in the CPU oracle run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-hhs", action="store_true")
    ap.add_argument("--no-chin", action="store_true",
                    help="skip the fourth-order integrator against KDK at equal cost")
    ap.add_argument("--no-reference", action="store_true",
                    help="skip the high-accuracy reference solve (errors over all particles)")
    ap.add_argument("--no-inflight", action="store_true",
                    help="skip the leg with two independent solves in flight")
    ap.add_argument("--classic", action="store_true",
                    help="time the headline solves with the classic build sequence (three "
                         "header readbacks) instead of level prediction")
    ap.add_argument("--no-named", action="store_true",
                    help="skip the run at the workload's own parameters (p 4, theta 0.5, leaf 16)")
    ap.add_argument("--ensemble", type=int, default=512, metavar="K",
                    help="requests in the serving ensemble (0: skip; the full stream is 512)")
    ap.add_argument("--ensemble-t-end", type=float, default=1.0)
    ap.add_argument("--ensemble-load", type=float, default=0.7,
                    help="Poisson rate as a fraction of the closed-loop saturation rate")
    ap.add_argument("--ensemble-slots", type=int, default=256)
    ap.add_argument("--ensemble-arena-gib", type=int, default=16)
    ap.add_argument("--ensemble-max-n", type=int, default=1 << 22)
    ap.add_argument("--configs", type=int, nargs="*", default=[0, 1, 2, 3],
                    help="named workloads measured in the per-configuration leg")
    ap.add_argument("--no-configs", action="store_true")
    ap.add_argument("--collapse-t-end", type=float, default=0.25,
                    help="end time of the cold-collapse HHS run (two free-fall times: 2.2214)")
    ap.add_argument("--collapse-run", type=int, default=0, metavar="N",
                    help="only integrate a cold collapse of N particles to --collapse-t-end "
                         "(both precisions) and exit")
    ap.add_argument("--hhs-request", type=int, default=-1, metavar="I",
                    help="only time top-level HHS steps of ensemble request I (mixed, the "
                         "ensemble parameters) and exit; used for kernel traces of small systems")
    ap.add_argument("--hhs-steps", type=int, default=2)
    ap.add_argument("--hhs-leaf", type=int, default=0, help="leaf size of --hhs-request")
    ap.add_argument("--hhs-small-path", type=int, default=1, choices=(0, 1, 2),
                    help="single-workgroup builds in --hhs-request (fmm_set_small_path)")
    ap.add_argument("--hhs-predict", type=int, default=0, choices=(0, 1),
                    help="level prediction in --hhs-request (fmm_set_level_prediction)")
    ap.add_argument("--graph-ab", type=int, default=0, metavar="REPS",
                    help="only run the HIP-graph replay A/B of one evaluation (REPS repeats "
                         "each way) and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (3 times) and exit; used to "
                         "scale the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 3}))
        return
    if args.graph_ab:
        graph_ab_leg(args)
        return
    if args.hhs_request >= 0:
        hhs_request_leg(args)
        return
    if args.collapse_run > 0:
        collapse_run_leg(args)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the FMM solve here is a single-device path)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1712_10116_amd.fmm as F
    from paper_1712_10116_amd import autotune
    from paper_1712_10116_amd import workloads as W

    dev = torch.device("cuda:0")
    n = args.n
    eps = 0.005
    pos, vel, mass = W.uniform_sphere(n, seed=1001)
    tp = torch.from_numpy(pos).to(dev)
    tm = torch.from_numpy(mass).to(dev)
    line_tune = None
    if args.no_tune:
        prm = dict(p=args.p, theta=args.theta, eps=eps, leaf_size=args.leaf)
    else:
        progress("autotuner")
        t0 = time.perf_counter()
        tr = autotune.tune(tp, tm, eps=eps, kernel=F.WENDLAND, precision=F.MIXED,
                           target=args.target, leaf_sizes=(24, 32, 48, 64, 96, 128),
                           orders=(4, 5, 6), thetas=(0.4, 0.45, 0.5, 0.55, 0.6), reps=3)
        b = tr["best"]
        prm = dict(p=b["p"], theta=b["theta"], eps=eps, leaf_size=b["leaf_size"])
        ok = sorted((r for r in tr["table"] if r["ms"] is not None), key=lambda r: r["ms"])
        line_tune = {"target_rms": args.target, "candidates": len(tr["table"]),
                     "passing": len(ok), "seconds": round(time.perf_counter() - t0, 2),
                     "reference": tr["reference"],
                     "best": {k: (round(v, 6) if isinstance(v, float) else v) for k, v in b.items()},
                     "runners_up": [{k: (round(v, 6) if isinstance(v, float) else v)
                                     for k, v in r.items()} for r in ok[1:4]]}
    # the same (theta, p, leaf) for both precisions: equal truncation error
    # a steady loop over one system: the library's level prediction (tree and
    # walk queued for the split depth of the recent builds, one header
    # readback per solve) is on unless --classic; the classic sequence (three
    # readbacks) is timed beside it
    predict = not args.classic
    runs = [("mixed", F.MIXED, prm, predict), ("fp64", F.FP64, prm, predict)]
    if predict:
        runs.append(("mixed_classic", F.MIXED, prm, False))
    named = dict(p=4, theta=0.5, eps=eps, leaf_size=16)
    if not args.no_named and named != prm:
        runs.append(("mixed_named", F.MIXED, named, predict))
    res = {}
    for name, prec, pr, pred in runs:
        progress(f"timed solves: {name}")
        s = F.Solver(n, p_max=pr["p"], leaf_size=pr["leaf_size"], kernel=F.WENDLAND,
                     precision=prec)
        s.set_level_prediction(pred)
        acc = torch.empty((3, n), dtype=torch.float64, device=dev)
        pot = torch.empty((n,), dtype=torch.float64, device=dev)
        sec, phases, kt = time_solver(F, torch, s, tp, tm, acc, pot, pr, args.steps,
                                      args.warmup, profile=True)
        info = s.tree_info()
        inv = s.invariants(mass=tm, acc=acc)
        res[name] = dict(sec=sec, phases=phases, kt=kt, info=info, acc=acc.cpu().numpy(), prm=pr,
                         momentum=float(np.abs(inv["F"]).max() / inv["Fabs"]))
        s.close()
        del acc, pot
        torch.cuda.synchronize()
    # force error of every run over all particles against a high-accuracy
    # FP64 solve of the same particles
    rp = autotune.REFERENCE
    a_ref = None
    if not args.no_reference:
        s = F.Solver(n, p_max=rp["p"], leaf_size=rp["leaf_size"], kernel=F.WENDLAND,
                     precision=F.FP64)
        a_ref, _ = s.forces(tp, tm, eps=eps, theta=rp["theta"], p=rp["p"])
        a_ref = a_ref.cpu().numpy()
        s.close()

    mixed, fp64 = res["mixed"], res["fp64"]
    e_mf = force_error(mixed["acc"], fp64["acc"])
    ph = mixed["phases"]
    info = mixed["info"]
    steps = args.steps
    # dominant evaluation kernel and its algorithmic work per launch; launch
    # durations from the events around the two kernels in the timed region
    kern = {}
    kt = mixed["kt"]
    p2p_ms = kt["p2p"][0] / max(kt["p2p"][1], 1)
    m2l_ms = kt["m2l"][0] / max(kt["m2l"][1], 1)
    p2p_flops = P2P_FLOPS_PER_PAIR * info["p2p_interactions"] / 2.0
    m2l_flops = m2l_flops_per_pair(prm["p"]) * info["m2l"]
    kern["p2p"] = dict(ms=p2p_ms, flops=p2p_flops, tflops=p2p_flops / (p2p_ms * 1e-3) / 1e12)
    kern["m2l"] = dict(ms=m2l_ms, flops=m2l_flops, tflops=m2l_flops / (m2l_ms * 1e-3) / 1e12)
    # the dominant kernel is the one with the most algorithmic work; M2L's
    # event interval overlaps P2P (both run at once on two streams), so event
    # durations would not rank them
    dom = max(kern, key=lambda k: kern[k]["flops"])
    roof = dict(kernel=dom, bound="alu", achieved=round(kern[dom]["tflops"], 3),
                peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                frac=round(kern[dom]["tflops"] / PEAK_FP32_TFLOPS, 4),
                traffic=recorded_traffic(dom, prm))

    line = {
        "metric": METRIC,
        "value": round(n / mixed["sec"], 1),
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(mixed["sec"] * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"cold collapse, uniform unit sphere, N={n}, Wendland C2 "
                               f"eps={eps}, p={prm['p']}, theta={prm['theta']}, leaf "
                               f"{prm['leaf_size']} (autotuned for rms force error <= "
                               f"{args.target}), mixed FP32/FP64",
                   "n": n, "p": prm["p"], "theta": prm["theta"], "eps": eps,
                   "leaf_size": prm["leaf_size"], "level_prediction": predict,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "force_err": {"mixed_vs_fp64_gpu": {"rms": e_mf[0], "p99": e_mf[1]},
                      "vs_reference_all": {}, "vs_direct_sample": {},
                      "reference": dict(rp, precision="fp64")},
        "fp64": {"value": round(n / fp64["sec"], 1), "ms_per_step": round(fp64["sec"] * 1e3, 4),
                 "phases_ms": {k: round(v[0] / steps, 4) for k, v in fp64["phases"].items()}},
        "momentum_rel": {"mixed": mixed["momentum"], "fp64": fp64["momentum"]},
        "classic_sequence": ({"value": round(n / res["mixed_classic"]["sec"], 1),
                              "ms_per_step": round(res["mixed_classic"]["sec"] * 1e3, 4)}
                             if "mixed_classic" in res else None),
        "phases_ms": {k: round(v[0] / steps, 4) for k, v in ph.items()},
        "kernels": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in d.items()}
                    for k, d in kern.items()},
        "tree": info,
        "interactions_per_s": {"p2p_ordered": round(info["p2p_interactions"] / mixed["sec"], 1),
                               "m2l_ordered": round(info["m2l_directed"] / mixed["sec"], 1)},
    }
    for name, r in res.items():
        if a_ref is not None:
            e = force_error(r["acc"], a_ref)
            line["force_err"]["vs_reference_all"][name] = {"rms": e[0], "p99": e[1]}
    if line_tune:
        line["autotune"] = line_tune

    # two independent solves in flight: two contexts on two streams, called
    # alternately, so that one solve's latency-bound build (sort, tree, walk)
    # runs beside the other's evaluation (serving-style throughput; each call
    # is still one complete solve)
    if not args.no_inflight:
        progress("two solves in flight")
        sa = torch.cuda.Stream()
        sb = torch.cuda.Stream()
        pair = []
        for st in (sa, sb):
            with torch.cuda.stream(st):
                sv = F.Solver(n, p_max=prm["p"], leaf_size=prm["leaf_size"], kernel=F.WENDLAND,
                              precision=F.MIXED, stream=st)
                sv.set_level_prediction(predict)
                pair.append((sv, st, torch.empty((3, n), dtype=torch.float64, device=dev),
                             torch.empty((n,), dtype=torch.float64, device=dev)))
        kw2 = dict(eps=eps, theta=prm["theta"], p=prm["p"])
        torch.cuda.synchronize()
        for sv, st, a2, p2 in pair:
            with torch.cuda.stream(st):
                sv.forces(tp, tm, acc=a2, pot=p2, **kw2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(2 * args.steps):
            sv, st, a2, p2 = pair[k % 2]
            with torch.cuda.stream(st):
                sv.forces(tp, tm, acc=a2, pot=p2, **kw2)
        torch.cuda.synchronize()
        sec2 = (time.perf_counter() - t0) / (2 * args.steps)
        same = bool(torch.equal(pair[0][2], pair[1][2]))
        for sv, *_ in pair:
            sv.close()
        line["two_in_flight"] = {"solves": 2 * args.steps, "ms_per_solve": round(sec2 * 1e3, 4),
                                 "particles_per_s": round(n / sec2, 1),
                                 "results_equal": same, "precision": "mixed"}

    # force gradient d a_i/d x_i beside the forces (the input of the fourth-order
    # integrator the paper proposes in Sec. 4.1), same particles and parameters
    progress("force gradient")
    s = F.Solver(n, p_max=prm["p"], leaf_size=prm["leaf_size"], kernel=F.WENDLAND,
                 precision=F.MIXED)
    kw = dict(eps=eps, theta=prm["theta"], p=prm["p"])
    s.forces_grad(tp, tm, **kw)
    reps = 5
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        s.forces_grad(tp, tm, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        s.forces(tp, tm, **kw)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    line["force_gradient"] = {"ms_forces_and_gradient": round((t1 - t0) / reps * 1e3, 3),
                              "ms_forces": round((t2 - t1) / reps * 1e3, 3), "precision": "mixed"}
    s.close()

    if not args.no_hhs:
        progress("HHS step")
        # one HHS top-level step of the same particles (mixed precision)
        s = F.Solver(n, p_max=prm["p"], leaf_size=prm["leaf_size"], kernel=F.WENDLAND,
                     precision=F.MIXED)
        tpp = tp.clone()
        tv = torch.from_numpy(vel).to(dev)
        h = F.HHS(s, tpp, tv, tm, eps=eps, theta=prm["theta"], p=prm["p"], eta=0.0025,
                  max_levels=10)
        h.init()
        dtmax = float(np.sqrt(0.0025 * eps / max(float(h.a_cur[h.a_cur > 0].min()), 1e-30)))
        dt_top = min(2.0 ** np.floor(np.log2(dtmax)), 2.0 ** -4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = h.step(dt_top)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rungs = torch.bincount(h.rung.long()).cpu().numpy().tolist()
        # momentum change over the step, against sum m |a| dt_top (FP64 acc of the timed solves)
        a64 = res["fp64"]["acc"]
        p_scale = float((mass * np.sqrt((a64 * a64).sum(axis=0))).sum()) * dt_top
        P0 = (mass * vel).sum(axis=1)

        def dp(pp, vv):
            return float(np.abs(s.invariants(pos=pp, vel=vv, mass=tm)["P"] - P0).max() / p_scale)

        line["hhs"] = {"dt_top": dt_top, "seconds": round(t1 - t0, 4), **st,
                       "particles_per_s": round(st["force_particles"] / (t1 - t0), 1),
                       "rung_histogram": rungs, "momentum_change": dp(tpp, tv)}
        # the same step with the total-acceleration bound of Eq. 9 (eta1 = eta)
        progress("HHS step with the Eq. 9 bound")
        tpp = tp.clone()
        tv = torch.from_numpy(vel).to(dev)
        h = F.HHS(s, tpp, tv, tm, eps=eps, theta=prm["theta"], p=prm["p"], eta=0.0025,
                  max_levels=10, eta1=0.0025)
        h.init()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = h.step(dt_top)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        line["hhs_eq9"] = {"dt_top": dt_top, "eta1": 0.0025, "seconds": round(t1 - t0, 4), **st,
                           "particles_per_s": round(st["force_particles"] / (t1 - t0), 1),
                           "rung_histogram": torch.bincount(h.rung.long()).cpu().numpy().tolist(),
                           "momentum_change": dp(tpp, tv)}
        # the same particles stepped in comoving form (Sec. 3.5): flat LambdaCDM
        # (0.3, 0.7, H0 = 1 in the time unit), one top step of dt_top in ln a from
        # a = 0.5, kicks and drifts scaled by the tabulated factors of Eqs. 10-11
        progress("HHS step, comoving form")
        tab = F.Cosmology(omega_m=0.3, omega_l=0.7, h0=1.0, a_min=0.1, a_max=2.0, n=2048)
        tpp = tp.clone()
        tv = torch.from_numpy(vel).to(dev)
        h = F.HHS(s, tpp, tv, tm, eps=eps, theta=prm["theta"], p=prm["p"], eta=0.0025,
                  max_levels=10, cosmo=tab, t=float(np.log(0.5)))
        h.init()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = h.step(dt_top)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        line["hhs_comoving"] = {"a_start": 0.5, "dlna_top": dt_top, "omega_m": 0.3,
                                "omega_l": 0.7, "seconds": round(t1 - t0, 4), **st,
                                "particles_per_s": round(st["force_particles"] / (t1 - t0), 1),
                                "rung_histogram":
                                    torch.bincount(h.rung.long()).cpu().numpy().tolist(),
                                "momentum_change": dp(tpp, tv)}
        tab.close()
        # the paper's comparison integrator (individual timesteps, Sec. 2.3) on
        # the same particles and top step: 1 + 2^R all-particle solves
        progress("individual-timestep step")
        tpp = tp.clone()
        tv = torch.from_numpy(vel).to(dev)
        g = F.HHS(s, tpp, tv, tm, eps=eps, theta=prm["theta"], p=prm["p"], eta=0.0025,
                  max_levels=10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = g.trad_step(dt_top)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        line["trad"] = {"dt_top": dt_top, "seconds": round(t1 - t0, 4), **st,
                        "particles_per_s": round(st["force_particles"] / (t1 - t0), 1),
                        "solves_per_s": round(st["force_calls"] / (t1 - t0), 1),
                        "rung_histogram": torch.bincount(g.rung.long()).cpu().numpy().tolist(),
                        "momentum_change": dp(tpp, tv)}
        s.close()

    if not args.no_chin:
        progress("fourth-order integrator against KDK")
        chin_leg(args, F, torch, line)

    if "mixed_named" in res:
        r = res["mixed_named"]
        line["named_config"] = {**{k: v for k, v in r["prm"].items() if k != "eps"},
                                "value": round(n / r["sec"], 1),
                                "ms_per_step": round(r["sec"] * 1e3, 4)}

    if args.ensemble > 0:
        progress("serving ensemble")
        ensemble_leg(args, F, torch, line)

    if not args.no_configs:
        configs_leg(args, F, torch, line)

    if not args.no_cpu_baseline:
        progress("CPU oracle")
        cpu_leg(args, n, pos, mass, res, prm, line)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
