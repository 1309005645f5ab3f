#!/usr/bin/env python
"""Throughput of the full coupled step (EK + LB + moving charged spheres) on one
MI355X, in million lattice-cell updates per second (MLUPS).

Default workload: 256^3 periodic box (16.8 M cells), FP32 storage with
deviations, 64 free charged spheres (R = 6, Z = +40), two monovalent species at
0.01, E = 0.01 along x -- the size at which the working set (~3.6 GB) exceeds
the 256 MB Infinity Cache, so that bandwidths are HBM bandwidths.  The same
workload is also timed in FP64 plain storage and the FP32/FP64 speedup
reported.  Inputs are seeded and synthetic (workloads.py) and resident in HBM
before the timed region.

One JSON line is printed with the contract fields plus:
  roofline      -- the dominant kernel (LB stream/collide): algorithmic bytes
                   per launch / its mean duration from HIP events on the
                   library's stream, against the 8 TB/s HBM peak; traffic =
                   HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE
                   counter passes stored by paper_1607_04572_amd/counters.py,
                   null once the kernel's sources differ from the measured ones;
  cpu_baseline  -- the FP64 CPU oracle timed on a few full steps (about 12 s)
                   of the same workload;
  ek_alu        -- the FP32 EK kernel, bound by its vector ALU work: VALU
                   instructions per launch from the stored SQ counter pass /
                   its mean duration, against the issue peak (null once its
                   sources differ from the measured ones);
  step_hbm      -- the whole FP32 step: HBM bytes of its kernels from the same
                   counter passes / the step time, against 8 TB/s (null once
                   any kernel source differs from the measured one);
  effective     -- the state floor (populations and densities read and
                   written once, potential once each way) x MLUPS, vs 8 TB/s;
  kernels       -- per-stage mean times and algorithmic-byte bandwidths;
                   particle_frac: the particle stages' share of the step;
  boundary_cost -- step time with the spheres moving vs the same geometry
                   fixed (static walls and charge), and partial-volume vs
                   simple scheme, beside the paper's +2 % and < 10 %;
  fp64_plain    -- the same workload in FP64;
  serve         -- the serving loop: 200 seeded requests (box edge 32-128,
                   1-16 spheres, 1000 steps each) arriving as a Poisson stream
                   at 0.8 x the capacity measured on a saturated batch of 40;
                   p50/p99 latency and aggregate MLUPS; the same stream at
                   2 x capacity (overload) under "at_load_2".
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Vector ALU issue peak: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 instruction per SIMD every 4 cycles (16 lanes
# per SIMD; 39.3 T lane operations/s, 78.6 TFLOP/s of unpacked FP32 FMA -- half the packed 157.3).
VALU_PEAK_GIPS = 256 * 4 * 2.4 / 4
METRIC = "EK MLUPS + % HBM roofline, FP32 vs FP64 plain; p50/p99 latency in serve loop"


def algorithmic_bytes(stage: str, w, elem: int, fused: bool = False) -> float:
    """Minimal HBM bytes per cell of one launch of a stage's kernels."""
    ns = len(w.species)
    nx = w.shape[0]
    h = (nx // 2 + 1) / nx  # half-spectrum cells per real cell
    cpx = 2 * elem
    if stage == "lb":
        # read and write 19 populations, read the force density, write the velocity, read the flag
        return 19 * elem * 2 + 3 * elem + 3 * elem + 1
    if stage == "ek" and not fused:
        # read densities, potential, Psi (float), velocity, flag; write densities and force
        return ns * elem + elem + 4 + 3 * elem + 1 + ns * elem + 3 * elem
    if stage == "ek":
        # fused EK + LB pass: the above plus 19 populations read and written and the velocity written
        return ns * elem + elem + 4 + 3 * elem + 1 + ns * elem + 3 * elem + 19 * elem * 2 + 3 * elem
    if stage == "poisson":
        # X: read densities + particle charge, write half spectrum; Y, Z(+inverse), Y':
        # read + write it; X': read it, write phi
        return (ns * elem + elem + h * cpx) + 3 * 2 * h * cpx + (h * cpx + elem)
    return 0.0


def state_bytes(w, elem: int) -> int:
    """Bytes per lattice update that any implementation must move: the 19
    populations and n_s densities read and written once, the potential written
    and read once."""
    return 2 * (19 + len(w.species)) * elem + 2 * elem


def run_gpu(w, steps: int, warmup: int, profile_steps: int):
    import numpy as np  # noqa: F401
    import torch

    from paper_1607_04572_amd import workloads as W
    from paper_1607_04572_amd.ek import EkSim

    rho0 = W.initial_densities(w)
    sim = EkSim(w, initial_density=rho0)
    sim.prepare()
    sim.step(warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stages = sim.profile(profile_steps)
    diag = sim.diagnostics()
    sim.close()
    del sim
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return dt, stages, diag


PARTICLE_STAGES = ("move", "geometry", "boundary", "forces", "finish")


def boundary_cost(w, steps: int, warmup: int) -> dict:
    """Cost of the moving boundaries, beside the paper's figures (Sec. IV.A):
    step time with the spheres moving vs the same geometry held fixed (the
    boundary cells and particle charge of the first step as static walls and
    static charge: no particle work), and with the partial-volume scheme vs
    the simple one.  The three runs are timed alike, one after the other."""
    import torch

    from paper_1607_04572_amd.ek import EkSim

    def timed(sim):
        sim.prepare()
        sim.step(warmup)
        sim.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        sim.sync()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        sim.close()
        torch.cuda.synchronize()
        return ms

    probe = EkSim(w, seeded=True)
    probe.prepare()
    mask, charge = probe.field("flag"), probe.field("particle_charge")
    probe.close()
    t_move = timed(EkSim(w, seeded=True))
    t_fixed = timed(EkSim(w.replace(spheres=[]), seeded=True, static_mask=mask, static_charge=charge))
    t_simple = timed(EkSim(w.replace(scheme="simple"), seeded=True))
    torch.cuda.empty_cache()
    return {"steps": steps, "moving_ms": t_move, "fixed_ms": t_fixed, "simple_ms": t_simple,
            "moving_over_fixed": t_move / t_fixed, "pv_over_simple": t_move / t_simple,
            "paper": {"moving_over_fixed": 1.02, "pv_over_simple_below": 1.10}}


def copy_probe(mib: int, reps: int = 10) -> dict:
    """Plain device copy of `mib` MiB (the library's copy kernel), timed with
    HIP events: the achievable streaming bandwidth, and a kernel of known
    traffic (mib MiB read + mib MiB written per launch) for scaling counters."""
    import torch

    from paper_1607_04572_amd.ek import ek_copy_probe
    n = mib * (1 << 20)
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty(n, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    st = torch.cuda.current_stream()
    ek_copy_probe(b.data_ptr(), a.data_ptr(), n, st.cuda_stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        ek_copy_probe(b.data_ptr(), a.data_ptr(), n, st.cuda_stream)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"bytes_per_launch": 2 * n, "ms": ms, "GBps": 2 * n / (ms * 1e-3) / 1e9}


def cpu_baseline(w, budget_s: float = 12.0, threads: int = 0) -> dict:
    """The FP64 CPU oracle on a bounded sample of the same workload: full
    steps until about budget_s seconds have passed (2 to 8 steps), on
    `threads` OpenMP threads (0: as many as the environment gives)."""
    import ctypes

    from oracle import oracle as O
    from paper_1607_04572_amd import workloads as W

    if threads > 0:
        O.lib().or_set_num_threads(ctypes.c_int(threads))

    p = O.make_params(*w.shape, w.nu, w.kT, w.lambda_B, w.E, [(s.D, s.z) for s in w.species],
                      partial_volume=w.scheme == "pv", charge_mode=1 if w.charge == "uniform" else 0,
                      integrator=0 if w.integrator == "vv" else 1)
    spheres = [dict(x=s.x, R=s.R, Z=s.Z, M=s.M, v=s.v, mode=s.mode) for s in w.spheres]
    o = O.OracleSim(p, spheres, W.initial_densities(w))
    o.step()  # first step outside the sample (page-in of the fields)
    n, dt = 0, 0.0
    t0 = time.perf_counter()
    while n < 8 and (n < 2 or dt < budget_s):
        o.step()
        n += 1
        dt = time.perf_counter() - t0
    lib = O.lib()
    lib.or_num_threads.restype = ctypes.c_int
    threads = int(lib.or_num_threads())
    return {"value": w.cells * n / dt / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{n} full steps of {w.name} ({w.cells} cells, FP64 oracle) after one untimed, {dt:.1f} s"}


def progress(msg: str):
    """One line per finished stage on stderr (a long run shows it is alive)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c3", choices=["c0", "c1", "c2", "c3"])
    ap.add_argument("--profile-steps", type=int, default=10)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-boundary-cost", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0, help="threads of the CPU oracle (0: all it is given)")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run the plain copy kernel on buffers of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the library has no multi-GPU "
              "path: the domain decomposition is described, not implemented.", file=sys.stderr)
        sys.exit(2)

    from paper_1607_04572_amd import workloads as W

    w32 = W.CONFIGS[args.workload]("fp32") if args.workload != "c0" else W.c0()
    dt, stages, diag = run_gpu(w32, args.steps, args.warmup, args.profile_steps)
    mlups = w32.cells * args.steps / dt / 1e6
    progress(f"{w32.name}: {mlups:.0f} MLUPS")
    fp64 = w32.precision == "fp64"  # the 32^3 prescribed-sphere case: FP64 plain, EK and LB fused
    elem = 8 if fp64 else 4
    kern = {}
    for st in (("ek", "poisson") if fp64 else ("lb", "ek", "poisson")):
        bpc = algorithmic_bytes(st, w32, elem, fused=fp64 and st == "ek")
        ms = stages[st]
        kern[st] = {"ms": ms, "GBps": bpc * w32.cells / (ms * 1e-3) / 1e9, "bytes_per_cell": bpc}
    fk = kern["ek" if fp64 else "lb"]
    from paper_1607_04572_amd import counters
    meas = None if fp64 else counters.stored_traffic()
    lb_bytes = fk["bytes_per_cell"] * w32.cells
    out = {
        "metric": METRIC, "value": mlups, "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": w32.precision, "data": "synthetic",
        "config": {"workload": w32.name, "cells": w32.cells, "shape": list(w32.shape),
                   "spheres": len(w32.spheres), "species": len(w32.species),
                   "storage": "fp64 plain" if fp64 else "fp32 deviations (fp64 particles, sums, redistribution)",
                   "scheme": "partial volume" if w32.scheme == "pv" else "simple", "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": "k_ek (EK + LB fused)" if fp64 else "k_lb (stream/collide)",
                     "achieved": fk["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": fk["GBps"] / HBM_PEAK_GBS,
                     "traffic": meas["traffic_bytes_per_launch"] if meas else None,
                     "traffic_over_algorithmic": meas["traffic_bytes_per_launch"] / lb_bytes if meas else None,
                     "bytes_per_launch": lb_bytes, "launch_ms": fk["ms"]},
        # the state floor: populations and densities read and written once, the potential once each way
        "effective": {"bytes_per_lup": state_bytes(w32, elem), "GBps": state_bytes(w32, elem) * mlups * 1e6 / 1e9,
                      "frac": state_bytes(w32, elem) * mlups * 1e6 / 1e9 / HBM_PEAK_GBS},
        # the whole step from the stored counter passes: HBM bytes of its kernels / the step time
        "step_hbm": None if fp64 or counters.stored_step_bytes() is None else {
            "bytes_per_step": counters.stored_step_bytes(),
            "GBps": counters.stored_step_bytes() / (dt / args.steps) / 1e9,
            "frac": counters.stored_step_bytes() / (dt / args.steps) / 1e9 / HBM_PEAK_GBS},
        "ek_alu": None if fp64 or counters.stored_valu() is None else {
            "bound": "alu", "kernel": "k_ek32 (EK, FP32)", "unit": "G wave64 VALU instructions/s",
            "achieved": counters.stored_valu()["valu_per_launch"] / (stages["ek"] * 1e-3) / 1e9,
            "peak": VALU_PEAK_GIPS,
            "frac": counters.stored_valu()["valu_per_launch"] / (stages["ek"] * 1e-3) / 1e9 / VALU_PEAK_GIPS,
            "valu_per_launch": counters.stored_valu()["valu_per_launch"], "launch_ms": stages["ek"]},
        "kernels": {"stage_ms": stages, **{k: v for k, v in kern.items()},
                    "particle_frac": sum(stages[k] for k in PARTICLE_STAGES) / sum(stages.values())},
        "diagnostics": {"species_total": [float(x) for x in diag["species_total"][:len(w32.species)]],
                        "max_velocity": diag["max_velocity"]},
    }
    if not args.no_boundary_cost:
        out["boundary_cost"] = boundary_cost(w32, min(args.steps, 100), args.warmup)
        progress("boundary cost done")
    if not args.no_fp64 and not fp64:
        w64 = w32.replace(precision="fp64", name=w32.name.replace("fp32", "fp64"))
        steps64 = max(10, args.steps // 2)
        dt64, st64, _ = run_gpu(w64, steps64, args.warmup, args.profile_steps)
        m64 = w64.cells * steps64 / dt64 / 1e6
        b64 = algorithmic_bytes("ek", w64, 8, fused=True) * w64.cells
        out["fp64_plain"] = {"value": m64, "unit": "MLUPS", "ms_per_step": dt64 / steps64 * 1e3,
                             "steps": steps64, "stage_ms": st64,
                             "fused_ek_lb_GBps": b64 / (st64["ek"] * 1e-3) / 1e9}
        out["fp32_over_fp64"] = mlups / m64
        progress(f"fp64: {m64:.0f} MLUPS")
    if not args.no_serve:
        from paper_1607_04572_amd import serve
        out["serve"] = serve.serve_benchmark(n_requests=args.serve_requests, extra_loads=(2.0,))
        progress("serve loop done")
    if args.copy_probe_mib:
        out["copy_probe"] = copy_probe(args.copy_probe_mib)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w32, threads=args.cpu_threads)
        progress("cpu baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
