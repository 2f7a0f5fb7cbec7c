"""Open- and closed-loop drivers of the request server (``fmm.Server``).

The server (native code behind serve_* in the C ABI) does the admission,
batching and stepping; these helpers only feed it requests at their arrival
times and collect what it returns, so that latency can be measured.
"""
from __future__ import annotations

import time

import numpy as np


def poisson_arrivals(n, rate, seed):
    """Arrival times (seconds from the start) of n requests of a Poisson
    process with the given rate (per second)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))


def run(server, requests, t_end, arrivals=None, clock=time.perf_counter, log=None):
    """Serve ``requests`` (a list of (pos, vel, mass) host arrays) to ``t_end``.

    arrivals: seconds after the start at which request k arrives (None: all at
    once, a closed loop).  Returns (results, makespan): one dict per request in
    request order, with the server's result fields, the final pos/vel, and
    ``latency`` = completion time minus arrival time (a request that arrives
    while the server is stepping is handed over when the step ends, and that
    wait counts too), and the time from the start to the last completion."""
    n = len(requests)
    arr = np.zeros(n) if arrivals is None else np.asarray(arrivals, dtype=np.float64)
    order = np.argsort(arr, kind="stable")
    nxt = 0
    ids = {}
    results = [None] * n
    start = clock()
    outstanding = 0
    steps = 0
    last_log = -1e9
    while nxt < n or outstanding:
        now = clock() - start
        while nxt < n and arr[order[nxt]] <= now:
            k = int(order[nxt])
            pos, vel, mass = requests[k]
            rid = server.submit(pos, vel, mass, t_end)
            ids[rid] = (k, clock() - start)
            outstanding += 1
            nxt += 1
        if outstanding:
            nr, nq = server.step()
            steps += 1
            if log is not None and clock() - last_log >= 2.0:   # a line every 2 s at most
                last_log = clock()
                log(f"step {steps}: {nr} resident, {nq} queued, {last_log - start:.1f} s")
            for r in server.poll():
                k, t_sub = ids.pop(r["id"])
                # server clock: t_done - t_submit; driver clock: hand-over delay
                r["latency"] = (t_sub - arr[k]) + (r["t_done"] - r["t_submit"])
                r["arrival"] = float(arr[k])
                r["done"] = t_sub + (r["t_done"] - r["t_submit"])
                results[k] = r
                outstanding -= 1
        elif nxt < n:
            time.sleep(max(0.0, arr[order[nxt]] - (clock() - start)))
    makespan = max(r["done"] for r in results) if n else 0.0
    return results, makespan


def summary(results, makespan):
    """Throughput and latency percentiles of one run."""
    lat = np.array([r["latency"] for r in results])
    parts = sum(r["force_particles"] for r in results)
    return dict(
        requests=len(results),
        makespan_s=makespan,
        requests_per_s=len(results) / makespan if makespan > 0 else None,
        particles_per_s=parts / makespan if makespan > 0 else None,
        force_particles=int(parts),
        p50_s=float(np.percentile(lat, 50)) if lat.size else None,
        p99_s=float(np.percentile(lat, 99)) if lat.size else None,
        max_s=float(lat.max()) if lat.size else None,
    )
