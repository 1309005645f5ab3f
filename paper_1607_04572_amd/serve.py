"""Continuous-batching serving loop for electrophoresis requests.

Requests (box, spheres, field, salt, steps) arrive on a seeded Poisson
process.  An arrived request is admitted into the device batch as soon as a
slot and a contiguous range of the arena of its footprint are free; all
admitted requests advance together in batched steps (one launch per kernel
for the whole mix, replayed from a HIP graph), and a request that has run its
steps is collected and its memory freed, which lets the next one in.
Reported: latency (completion - arrival) percentiles and aggregate MLUPS."""
from __future__ import annotations

import collections
import time

import numpy as np

from . import workloads as W
from .ek import EkBatch, EkError


def run(requests: list, arena_bytes: int = 24 << 30, chunk: int = 20, clock=time.perf_counter) -> dict:
    """requests: [(arrival_seconds, Workload)], sorted by arrival.

    A request's initial state (its seeded densities) is built on the device
    at admission, so the host does no per-cell work for it."""
    batch = EkBatch(arena_bytes, n_species=len(requests[0][1].species))
    pending = collections.deque((t, i, w) for i, (t, w) in enumerate(sorted(requests, key=lambda r: r[0])))
    arrival = {}
    latency = []
    lups = 0
    t0 = clock()
    done = 0
    n_req = len(requests)
    max_active = 0
    failed = 0
    try:
        while done < n_req:
            now = clock() - t0
            # admit everything that has arrived, in order, while it fits
            while pending and pending[0][0] <= now:
                t_arr, i, w = pending[0]
                try:
                    slot = batch.admit(w, seeded=True)
                except EkError as e:
                    if e.code == -6:  # no slot or memory: wait for a completion
                        break
                    raise
                arrival[slot] = (t_arr, w)
                pending.popleft()
            n_act, _ = batch.active()
            max_active = max(max_active, n_act)
            if n_act:
                batch.step(chunk)
            elif pending:
                wait = pending[0][0] - (clock() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.01))
            for slot in batch.poll():
                t_arr, w = arrival.pop(slot)
                done += 1
                try:
                    batch.collect(slot)
                except EkError as e:
                    if e.code not in (-3, -7):  # unstable / non-finite: the request failed alone
                        raise
                    failed += 1
                    continue
                latency.append(clock() - t0 - t_arr)
                lups += w.cells * w.steps
        wall = clock() - t0
    finally:
        batch.close()
    lat = np.array(latency)
    return {"requests": n_req, "wall_s": wall, "mlups": lups / wall / 1e6,
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "max_active": max_active, "failed": failed}


def saturated_capacity(requests: list, arena_bytes: int = 24 << 30, chunk: int = 20) -> dict:
    """All requests available at t = 0: the batch stays as full as memory and
    slots allow.  Returns throughput and requests per second."""
    reqs = [(0.0, w) for _, w in requests]
    r = run(reqs, arena_bytes, chunk)
    r["req_per_s"] = len(reqs) / r["wall_s"]
    return r


def serve_benchmark(n_requests: int = 200, seed: int = 1611, load: float = 0.8, n_calibrate: int = 40,
                    steps: int = 1000, arena_bytes: int = 24 << 30, extra_loads: tuple = ()) -> dict:
    """Measure the saturated capacity on the first n_calibrate requests of the
    stream, then serve n_requests arriving at load * capacity.  Each entry of
    extra_loads serves the same stream again at that multiple of the capacity
    (e.g. 2.0: overload) and is reported under "at_load_<x>"."""
    calib = W.serve_requests(n_calibrate, seed=seed, rate=1.0, steps=steps)
    cap = saturated_capacity(calib, arena_bytes)
    out = None
    for i, ld in enumerate((load,) + tuple(extra_loads)):
        rate = ld * cap["req_per_s"]
        reqs = W.serve_requests(n_requests, seed=seed, rate=rate, steps=steps)
        res = run(reqs, arena_bytes)
        res.update({"rate_req_per_s": rate, "load": ld, "capacity_req_per_s": cap["req_per_s"],
                    "capacity_mlups": cap["mlups"], "seed": seed, "steps_per_request": steps})
        if i == 0:
            out = res
        else:
            out[f"at_load_{ld:g}"] = {k: res[k] for k in ("p50_s", "p99_s", "mean_s", "mlups", "max_active",
                                                          "rate_req_per_s", "wall_s")}
    return out
