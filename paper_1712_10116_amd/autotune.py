"""Autotuner for the force solve: picks the leaf size, opening angle and
expansion order that reach a force-error target fastest on a given particle
set and precision.

The error of a candidate is measured against a high-accuracy FP64 solve of the
same particles on the GPU (order 6, theta 0.25, large leaves), whose own error
is far below the targets of interest; the error of particle i is
|a_i - a_i^ref| / max(|a_i^ref|, 1e-6 rms|a^ref|) and a candidate passes when
the rms over the particles is within the target.  Every passing candidate is
timed (complete solve: box, keys, sort, tree, walk, evaluation; median of a
few calls after a warm-up) and the fastest wins.

The truncation error depends on (theta, p) and only weakly on the leaf size
(larger leaves move pairs from M2L to exact P2P), while the cost depends on
all three, so the search covers the full grid but skips the timing of
candidates that miss the target.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import fmm as F

LEAF_SIZES = (8, 16, 24, 32, 48, 64, 96, 128)
ORDERS = (3, 4, 5, 6)
THETAS = (0.3, 0.35, 0.4, 0.45, 0.5, 0.55)
REFERENCE = dict(p=6, theta=0.25, leaf_size=64)


def _rel_rms(acc, ref):
    mag = torch.linalg.vector_norm(ref, dim=0)
    floor = 1e-6 * torch.sqrt((mag * mag).mean())
    e = torch.linalg.vector_norm(acc - ref, dim=0) / torch.clamp(mag, min=float(floor))
    return float(torch.sqrt((e * e).mean()))


def _time(s, pos, mass, eps, theta, p, acc, pot, reps):
    s.forces(pos, mass, eps=eps, theta=theta, p=p, acc=acc, pot=pot)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        s.forces(pos, mass, eps=eps, theta=theta, p=p, acc=acc, pot=pot)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def tune(pos, mass, *, eps, kernel=F.WENDLAND, precision=F.MIXED, target=1e-3,
         leaf_sizes=LEAF_SIZES, orders=ORDERS, thetas=THETAS, reps=5, log=None):
    """Search (leaf_size, theta, p) for the fastest solve of (pos, mass) whose
    rms force error is at most ``target``.

    pos: device float64 (3, n); mass: device float64 (n,).  Returns a dict
    with the winner (leaf_size, theta, p, ms, err) and ``table``, one entry
    per candidate (ms is None for those that missed the target).  With
    target None every candidate is timed and no error is measured (for when
    theta and p are fixed by the caller and only the leaf size is free)."""
    n = pos.shape[1]
    dev = pos.device
    acc = torch.empty((3, n), dtype=torch.float64, device=dev)
    pot = torch.empty((n,), dtype=torch.float64, device=dev)
    a_ref = None
    if target is not None:
        ref = F.Solver(n, p_max=REFERENCE["p"], leaf_size=REFERENCE["leaf_size"], kernel=kernel,
                       precision=F.FP64)
        a_ref, _ = ref.forces(pos, mass, eps=eps, theta=REFERENCE["theta"], p=REFERENCE["p"])
        torch.cuda.synchronize()
        ref.close()
    table = []
    best = None
    for leaf in leaf_sizes:
        s = F.Solver(n, p_max=max(orders), leaf_size=leaf, kernel=kernel, precision=precision)
        for p in orders:
            for th in thetas:
                s.forces(pos, mass, eps=eps, theta=th, p=p, acc=acc, pot=pot)
                err = _rel_rms(acc, a_ref) if a_ref is not None else None
                ms = None
                if target is None or err <= target:
                    ms = 1e3 * _time(s, pos, mass, eps, th, p, acc, pot, reps)
                    if best is None or ms < best["ms"]:
                        best = dict(leaf_size=leaf, theta=th, p=p, ms=ms, err=err)
                table.append(dict(leaf_size=leaf, theta=th, p=p, err=err, ms=ms))
                if log:
                    log(table[-1])
        s.close()
    del a_ref
    return dict(best=best, table=table, target=target, n=n, eps=eps, kernel=kernel,
                precision=precision, reference=dict(REFERENCE))


def fastest(candidates, run, reps=2):
    """The candidate whose ``run(candidate)`` (returning seconds) is smallest,
    best of ``reps`` runs each, with the table of all timings.  Used where the
    cost is not a single solve, e.g. the leaf size of a request server, timed
    on a short closed-loop run of its own workload."""
    table = []
    for c in candidates:
        t = min(run(c) for _ in range(reps))
        table.append(dict(candidate=c, seconds=t))
    best = min(table, key=lambda r: r["seconds"])
    return dict(best=best["candidate"], table=table)
