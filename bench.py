"""Throughput benchmark of the USP-ESBGK particle step on one MI355X.

Workload (the paper's 1-D continuum cases at the sizes of the second
configuration): a thermal Couette flow and a Sod shock tube, each 1000 cells
x 500 particles per cell (FP32 state), Kn = 1e-3, dt = 5 mean collision
times, advanced together in the same kernel launches.  Synthetic inputs
(seeded Philox initial states); no external data.

A "step" is one full time step (Table 2 steps 2-8) of both instances.
value = live particles (weighted included) x steps / wall time of the timed
region, with all state resident in HBM.

Prints one JSON line (see the "roofline", "valu_issue" and "cpu_baseline"
members).
"""
import argparse
import hashlib

import numpy as np
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# algorithmic bytes per particle-step: one read and one write of the particle
# record (y, cx, cy, cz, w in FP32 = 20 B each way)
BYTES_PER_PARTICLE_STEP = 40.0
# algorithmic bytes per cell-step: Eq. 34 averages and J-moment averages read
# and written (2 x 2 x 13 FP64), moments and raw sums written (2 x 13 FP64),
# P_ne read (8 B), particle count written (4 B)
BYTES_PER_CELL_STEP = 6 * 13 * 8 + 8 + 4

# HBM traffic of the cell kernel measured by rocprofv3 (FETCH_SIZE,
# WRITE_SIZE) on this workload, with the hash of the kernel sources it was
# measured on: reported only while the sources are unchanged
PROFILE = os.path.join(ROOT, "profiles", "cell_kernel_thermal_couette_sod_1d.md")
KERNEL_SOURCES = ("usp_cell_impl.h", "usp_device.h", "usp_common.h", "usp_cell_f32_1d.hip",
                  "usp_kernels.hip")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1808_03801_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _profile_figure(key):
    """a per-step figure from the committed rocprofv3 summary, or None when
    it was taken on other kernel sources"""
    try:
        txt = open(PROFILE).read()
    except OSError:
        return None
    m = re.search(key + r":\s*([0-9.eE+]+)\s+sources:\s*([0-9a-f]+)", txt)
    if not m or m.group(2) != kernel_source_hash():
        return None
    return float(m.group(1))


def measured_traffic():
    """HBM bytes per step (FETCH_SIZE + WRITE_SIZE, copy-calibrated)"""
    return _profile_figure("traffic_bytes_per_step")


def measured_valu():
    """VALU wave instructions per step (SQ_INSTS_VALU over the step's dispatches)"""
    return _profile_figure("valu_instr_per_step")


# wave64 VALU instructions the chip can issue per second: 256 CUs x 4 SIMDs,
# one wave64 instruction per SIMD every 4 cycles (16 lanes), 2.4 GHz
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def copy_calibration():
    """a plain device copy of known size (256 MiB, three times), so that the
    FETCH_SIZE / WRITE_SIZE counters can be scaled to bytes"""
    import torch
    n = 64 * 1024 * 1024
    a = torch.ones(n, device="cuda", dtype=torch.float32)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": n * 4, "copies": 3}), flush=True)


def workload():
    from paper_1808_03801_amd import problems as P
    tc = P.thermal_couette_1d(Kn=1e-3, ncell=1000, ppc=500, dt_over_tau=5.0, seed=1)
    sod = P.sod_1d(Kn=1e-3, ncell=1000, mean_ppc=500, dt_over_tau=5.0, seed=2)
    return [tc, sod]


def cpu_baseline(steps=30):
    """the CPU oracle (single thread, as it stands) on the same two problems
    for a few steps from their initial state"""
    from oracle import oracle as O
    pbs = workload()
    os_ = [O.Oracle(pb) for pb in pbs]
    n0 = sum(o.num_particles() for o in os_)
    t0 = time.perf_counter()
    for _ in range(steps):
        for o in os_:
            o.step(1)
    dt = time.perf_counter() - t0
    n1 = sum(o.num_particles() for o in os_)
    return dict(value=0.5 * (n0 + n1) * steps / dt, unit="particle-updates/s", cores=1,
                kind="oracle",
                sample=f"{steps} steps of both instances from their initial state "
                       f"({n0}-{n1} live particles), {dt:.1f} s")


def serving(n, steps, budget):
    """The request mix of the serving workload (Poisson arrivals at 50/s,
    Couette / Poiseuille / Sod, Kn log-uniform in [1e-3, 1], 50-400 cells,
    50-200 particles per cell, steps uniform in `steps`), served with
    continuous batching and, for comparison, one request at a time."""
    import torch
    from paper_1808_03801_amd import serve as S
    from paper_1808_03801_amd import usp
    reqs = S.request_trace(n, rate=50.0, steps=steps, seed=0)
    ctx = usp.Context(0)
    srv = S.Server(ctx, budget=budget, chunk=50)
    futs = [srv.submit(r) for r in reqs]
    t0 = time.perf_counter()
    srv.run(t0=t0)
    wall_b = time.perf_counter() - t0
    batched = [f.result() for f in futs]
    t0 = time.perf_counter()
    plain = S.run_plain(ctx, reqs, t0=t0)
    wall_p = time.perf_counter() - t0
    same = all(
        np.array_equal(b.fields, p.fields)
        for b, p in zip(sorted(batched, key=lambda r: r.request.seed),
                        sorted(plain, key=lambda r: r.request.seed)))
    ctx.close()
    sb, sp = S.summarize(batched, wall_b), S.summarize(plain, wall_p)
    return {
        "requests": n, "steps_per_request": list(steps), "arrival_rate_per_s": 50.0,
        "hbm_budget_bytes": budget, "max_active": srv.max_active,
        "batched": sb, "plain": sp,
        "speedup_solves_per_s": sb["solves_per_s"] / sp["solves_per_s"],
        "results_identical_to_plain": bool(same),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--chunk", type=int, default=20, help="steps per library call")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--block", type=int, default=256)
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default launch shapes instead of autotuning them")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch eagerly instead of replaying captured HIP graphs")
    ap.add_argument("--serve", type=int, default=64,
                    help="requests of the serving measurement (0: skip it)")
    ap.add_argument("--serve-steps", default="200,1000",
                    help="step range of the serving requests (the full mix: 2000,10000)")
    ap.add_argument("--serve-budget", type=float, default=2.0, help="HBM budget, GiB")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see the design notes for how the step would shard)", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return

    import torch
    from paper_1808_03801_amd import usp

    pbs = workload()
    ctx = usp.Context(0)
    ctx.set_block(args.block)
    inst = [ctx.add(pb) for pb in pbs]
    ctx.set_graph(not args.no_graph)

    def run(n):
        left = n
        while left > 0:
            k = min(args.chunk, left)
            ctx.step(inst, k)
            left -= k

    run(args.warmup)
    ctx.sync()
    shapes = None
    if not args.no_tune:
        from paper_1808_03801_amd import autotune
        autotune.tune(ctx, inst, steps=5, repeats=2)
        shapes = {pb.name: i.shape()[0] for pb, i in zip(pbs, inst)}
        run(args.chunk)  # the tuned shapes' graphs are captured outside the timing
    ctx.sync()
    n_before = sum(i.num_particles() for i in inst)
    # GPU time of the timed region: HIP events on the library's stream (the
    # library works on torch's current stream) around the graph replays
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(ctx.stream)
    run(args.steps)
    ev1.record(ctx.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.sync()
    n_after = sum(i.num_particles() for i in inst)
    n_live = 0.5 * (n_before + n_after)
    value = n_live * args.steps / wall

    # one step = one cell-kernel pass (its launches over all shapes) plus the
    # P_ne and step-control kernels; the roofline prices the whole step's GPU
    # time, so the cell kernel's own rate is about 10 % higher
    step_ms = ev0.elapsed_time(ev1) / args.steps
    ncells = sum(pb.ncell for pb in pbs)
    bytes_per_step = n_live * BYTES_PER_PARTICLE_STEP + ncells * BYTES_PER_CELL_STEP
    achieved = bytes_per_step / (step_ms * 1e-3) / 1e9

    line = {
        "metric": "particle-updates/s",
        "value": value,
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "thermal Couette + Sod tube (1-D), 1000 cells x 500 particles/cell "
                        "each, Kn=1e-3, dt=5 tau_c, FP32 particles, FP64 cell moments, "
                        "both instances batched per launch",
            "cells": sum(pb.ncell for pb in pbs),
            "live_particles": int(n_live),
            "steps_per_call": args.chunk,
            "hip_graph": not args.no_graph,
            "first_launch_shape": shapes,
            "block": args.block,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "cell_kernel pass (fused relax + add + advect + bin) with the P_ne "
                      "and step-control kernels of the step",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": measured_traffic(),
            "avg_step_gpu_ms": step_ms,
            "bytes_per_step": bytes_per_step,
        },
    }
    # the same step seen from the vector ALUs: the kernel is bound by the
    # latency of its per-cell phases, and this says how busy the VALUs are
    valu = measured_valu()
    line["valu_issue"] = None if valu is None else {
        "instr_per_step": valu,
        "achieved": valu / (step_ms * 1e-3),
        "peak": VALU_ISSUE_PEAK,
        "unit": "wave64 VALU instructions/s",
        "frac": valu / (step_ms * 1e-3) / VALU_ISSUE_PEAK,
    }
    for i in inst:
        i.free()
    ctx.close()
    if args.serve > 0:
        lo, hi = (int(v) for v in args.serve_steps.split(","))
        line["serving"] = serving(args.serve, (lo, hi), int(args.serve_budget * (1 << 30)))
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
