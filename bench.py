"""Throughput benchmark of the USP-ESBGK particle step on one MI355X.

Headline workload (the largest single-GPU configuration): the flow through a
slit of Section 4.5, 400 x 200 cells, 100 particles per cell on average (8 M
per instance), pressure ratio 2, hard spheres, FP32 particle state with FP64
cell moments, at Kn = 0.01 and Kn = 0.1 -- both instances advanced together
in the same kernel launches (16.5 M live particles).  Further records: the
1-D thermal Couette flow and Sod tube of the continuum workload (1000 cells x
500 particles per cell each, Kn = 1e-3, dt = 5 tau_c) and the lid-driven
cavity of Section 4.4 (128 x 128 cells, 200 particles per cell, Kn = 1e-3,
1e-2 and 0.1 batched).  Serving: the request mix of Couette / Poiseuille / Sod
solves.  Synthetic inputs (seeded Philox initial states); no external data.

A "step" is one full time step (Table 2 steps 2-8) of every instance of the
workload.  value = live particles (weighted included) x steps / wall time of
the timed region, with all state resident in HBM.

Prints one JSON line (see the "roofline", "valu_issue", "c2", "c3", "serving"
and "cpu_baseline" members).
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def progress(msg):
    """one line on stderr as each phase of the run ends"""
    print("[bench] " + msg, file=sys.stderr, flush=True)


PEAK_HBM_GBS = 8000.0
# algorithmic bytes per particle-step: one read and one write of the particle
# record (FP32: y, cx, cy, cz, w = 20 B each way in 1-D; x as well in 2-D)
BYTES_PER_PARTICLE_STEP = {1: 40.0, 2: 48.0}
# algorithmic bytes per cell-step: Eq. 34 averages and J-moment averages read
# and written (2 x 2 x 13 FP64), moments and raw sums written (2 x 13 FP64),
# P_ne read (8 B), particle count written (4 B)
BYTES_PER_CELL_STEP = 6 * 13 * 8 + 8 + 4

# HBM traffic and VALU instructions of the step measured by rocprofv3 on each
# workload, with the hash of the kernel sources they were measured on: a
# figure is reported only while the sources are unchanged
PROFILES = {
    "c5": os.path.join(ROOT, "profiles", "cell_kernel_slit_2d_c5.md"),
    "c2": os.path.join(ROOT, "profiles", "cell_kernel_thermal_couette_sod_1d.md"),
    "c3": os.path.join(ROOT, "profiles", "cell_kernel_cavity_2d_c3.md"),
}
KERNEL_SOURCES = ("usp_cell_impl.h", "usp_device.h", "usp_common.h", "usp_cell_f32_1d.hip",
                  "usp_cell_f32_2d.hip", "usp_cell_f32_2d_xb.hip", "usp_kernels.hip")

# wave64 VALU instructions the chip can issue per second: 256 CUs x 4 SIMDs,
# one wave64 instruction per SIMD every 4 cycles (16 lanes), 2.4 GHz
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def _code_only(text):
    """source text without comments and blank lines (a comment cannot change
    a kernel, so it does not retire a measurement)"""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(l.rstrip() for l in text.splitlines() if l.strip())


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1808_03801_amd", "csrc", f)) as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def _profile_figure(workload, key):
    """a per-step figure from the committed rocprofv3 summary, or None when
    it was taken on other kernel sources"""
    try:
        txt = open(PROFILES[workload]).read()
    except (OSError, KeyError):
        return None
    m = re.search(key + r":\s*([0-9.eE+]+)\s+sources:\s*([0-9a-f]+)", txt)
    if not m or m.group(2) != kernel_source_hash():
        return None
    return float(m.group(1))


def regime_of(valu_frac, traffic_frac):
    """the regime, from the measured fractions of peak: the larger of VALU
    issue and measured HBM traffic (the algorithmic bytes are the roofline's
    floor, not a measurement of what the kernel moves)"""
    if valu_frac is not None and (traffic_frac is None or valu_frac >= traffic_frac):
        return "VALU issue and per-cell latency"
    if traffic_frac is not None:
        return "HBM traffic"
    return "unmeasured"


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


def workload_c5():
    """the slit of Section 4.5 at both Knudsen numbers (one instance each)"""
    from paper_1808_03801_amd import problems as P
    return [P.slit_2d(Kn=0.01, seed=1), P.slit_2d(Kn=0.1, seed=2)]


def workload_c2():
    from paper_1808_03801_amd import problems as P
    tc = P.thermal_couette_1d(Kn=1e-3, ncell=1000, ppc=500, dt_over_tau=5.0, seed=1)
    sod = P.sod_1d(Kn=1e-3, ncell=1000, mean_ppc=500, dt_over_tau=5.0, seed=2)
    return [tc, sod]


def workload_c3():
    """the lid-driven cavity of Section 4.4 at the three Knudsen numbers (one
    instance each, batched)"""
    from paper_1808_03801_amd import problems as P
    return [P.cavity_2d(Kn=kn, n=128, ppc=200, seed=11 + i)
            for i, kn in enumerate((1e-3, 1e-2, 0.1))]


WORKLOADS = {
    "c5": (workload_c5, "flow through a slit (2-D, Section 4.5), 400 x 200 cells, 100 "
                        "particles/cell mean (8 M per instance), pressure ratio 2, hard spheres, "
                        "Kn = 0.01 and Kn = 0.1 batched per launch, dt = 0.3 dx / mean speed, "
                        "FP32 particles, FP64 cell moments"),
    "c3": (workload_c3, "lid-driven cavity (2-D, Section 4.4), 128 x 128 cells, 200 "
                        "particles/cell (3.3 M per instance), lid 50 m/s, diffuse walls, "
                        "Kn = 1e-3, 1e-2 and 0.1 batched per launch, dt = 0.3 dx / mean speed, "
                        "FP32 particles, FP64 cell moments"),
    "c2": (workload_c2, "thermal Couette + Sod tube (1-D), 1000 cells x 500 particles/cell "
                        "each, Kn=1e-3, dt=5 tau_c, FP32 particles, FP64 cell moments, both "
                        "instances batched per launch"),
}


# ---- CPU baseline (the oracle as it stands) ---------------------------------

def _oracle_rate(name, steps, seed_offset=0):
    """one oracle instance of the workload's first problem: particle-updates
    per second over `steps` steps from the initial state"""
    from oracle import oracle as O
    pb = WORKLOADS[name][0]()[0]
    if seed_offset:
        pb = pb.replace(seed=pb.seed + seed_offset)
    o = O.Oracle(pb)
    n0 = o.num_particles()
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    n1 = o.num_particles()
    return 0.5 * (n0 + n1) * steps / dt, dt, n0


def _oracle_worker(args):
    return _oracle_rate(*args)


def cpu_baseline(name, steps):
    """The oracle (serial C, FP64, untuned) on the headline workload's first
    instance: one process on one core, then one process per host core (up
    to 16, the box's share) each stepping its own copy, summed.  Run before
    the GPU is touched (the worker processes are forked)."""
    import multiprocessing as mp
    one, dt1, n0 = _oracle_rate(name, steps)
    try:
        ncore = len(os.sched_getaffinity(0))
    except AttributeError:
        ncore = os.cpu_count() or 1
    ncore = max(1, min(ncore, 16))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(ncore) as pool:
        res = pool.map(_oracle_worker, [(name, steps, k + 1) for k in range(ncore)])
    wall = time.perf_counter() - t0
    allc = sum(r[0] for r in res)
    sample = (f"{steps} steps of the Kn = 0.01 slit (first instance of the workload, "
              f"{n0} particles) from its initial state: {dt1:.1f} s on one core; "
              f"{ncore} copies in parallel, {wall:.1f} s")
    return {"value": one, "unit": "particle-updates/s", "cores": 1, "kind": "oracle",
            "sample": sample,
            "all_cores": {"value": allc, "unit": "particle-updates/s", "cores": ncore,
                          "kind": "oracle", "sample": f"{ncore} processes, one copy each"}}


# ---- GPU measurement ---------------------------------------------------------

def measure(name, steps, warmup, chunk, graph, tune):
    """times `steps` steps of workload `name` (all its instances in every
    launch); returns the JSON members of that record"""
    import torch
    from paper_1808_03801_amd import usp
    builder, desc = WORKLOADS[name]
    pbs = builder()
    ctx = usp.Context(0)
    inst = [ctx.add(pb) for pb in pbs]
    ctx.set_graph(graph)

    def run(n):
        left = n
        while left > 0:
            k = min(chunk, left)
            ctx.step(inst, k)
            left -= k

    run(warmup)
    ctx.sync()
    tuned = None
    if tune:
        from paper_1808_03801_amd import autotune
        autotune.tune(ctx, inst, steps=5, repeats=2)
        run(chunk)  # the tuned shapes' graphs are captured outside the timing
    shapes = {pb.name + "_kn%g" % pb.meta["Kn"]: i.shape()[0] for pb, i in zip(pbs, inst)}
    ctx.sync()
    n_before = sum(i.num_particles() for i in inst)
    # GPU time of the timed region: HIP events on the library's stream (the
    # library works on torch's current stream) around the graph replays
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(ctx.stream)
    run(steps)
    ev1.record(ctx.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.sync()
    n_after = sum(i.num_particles() for i in inst)
    # real particles: the total weight (mass in units of N_p) of the instances
    real = sum(float(i.fields(0)[:, 0].sum()) for i in inst)
    for i in inst:
        assert i.status() == 0, (name, i.status())
    n_live = 0.5 * (n_before + n_after)
    # one step = one cell-kernel pass (its launches over all shapes) plus the
    # P_ne and step-control kernels; the roofline prices the whole step's GPU
    # time (an upper bound of the cell kernel's own time)
    step_ms = ev0.elapsed_time(ev1) / steps
    ncells = sum(pb.ncell for pb in pbs)
    dim = pbs[0].dim
    bytes_per_step = n_live * BYTES_PER_PARTICLE_STEP[dim] + ncells * BYTES_PER_CELL_STEP
    achieved = bytes_per_step / (step_ms * 1e-3) / 1e9
    traffic = _profile_figure(name, "traffic_bytes_per_step")
    valu = _profile_figure(name, "valu_instr_per_step")
    out = {
        "value": n_live * steps / wall,
        "real_particle_updates_per_s": real * steps / wall,
        "ms_per_step": wall / steps * 1e3,
        "config": {
            "workload": desc,
            "cells": ncells,
            "live_particles": int(n_live),
            "real_particles": int(round(real)),
            "steps_per_call": chunk,
            "hip_graph": graph,
            "first_launch_shape": shapes,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "cell_kernel pass (fused relax + add + advect + bin) with the P_ne "
                      "and step-control kernels of the step",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": traffic,
            "traffic_frac": (None if traffic is None
                             else traffic / (step_ms * 1e-3) / 1e9 / PEAK_HBM_GBS),
            "avg_step_gpu_ms": step_ms,
            "bytes_per_step": bytes_per_step,
        },
        # the same step seen from the vector ALUs: the cell kernel is bound by
        # the issue of its per-cell phases (much of it FP64), not by HBM
        "valu_issue": None if valu is None else {
            "instr_per_step": valu,
            "achieved": valu / (step_ms * 1e-3),
            "peak": VALU_ISSUE_PEAK,
            "unit": "wave64 VALU instructions/s",
            "frac": valu / (step_ms * 1e-3) / VALU_ISSUE_PEAK,
        },
    }
    r = out["roofline"]
    v = out["valu_issue"]
    vf = None if v is None else v["frac"]
    tf = r["traffic_frac"]
    regime = regime_of(vf, tf)
    r["regime"] = regime
    r["limiter"] = ("%s: VALU issue %s of peak, HBM %.1f %% of peak at the algorithmic "
                    "bytes and %s at the measured traffic"
                    % (regime, "unmeasured" if vf is None else "%.0f %%" % (100 * vf),
                       100 * r["frac"],
                       "unmeasured" if tf is None else "%.1f %%" % (100 * tf)))
    for i in inst:
        i.free()
    ctx.close()
    return out


def serving(n, steps, budget):
    """The request mix of the serving workload (Poisson arrivals at 50/s,
    Couette / Poiseuille / Sod, Kn log-uniform in [1e-3, 1], 50-400 cells,
    50-200 particles per cell, steps uniform in `steps`), served with
    continuous batching and, for comparison, one request at a time."""
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
    progress(f"serving: {n} requests batched in {wall_b:.1f} s")
    t0 = time.perf_counter()
    plain = S.run_plain(ctx, reqs, t0=t0)
    wall_p = time.perf_counter() - t0
    progress(f"serving: {n} requests one at a time in {wall_p:.1f} s")
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
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--chunk", type=int, default=20, help="steps per library call")
    ap.add_argument("--workload", default="c5", choices=sorted(WORKLOADS))
    ap.add_argument("--also", default="c2,c3",
                    help="workloads of the further records, comma-separated ('' for none)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default launch shapes instead of autotuning them")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch eagerly instead of replaying captured HIP graphs")
    ap.add_argument("--serve", type=int, default=256,
                    help="requests of the serving measurement (0: skip it)")
    ap.add_argument("--serve-steps", default="2000,10000",
                    help="step range of the serving requests")
    ap.add_argument("--serve-budget", type=float, default=2.0, help="HBM budget, GiB")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the step would shard by cell slabs or tiles per GPU, exchanging the "
              "particles that cross a shard boundary each step)", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return

    # the oracle first, in forked processes, before anything touches the GPU
    cpu = None if args.no_cpu else cpu_baseline(args.workload, args.cpu_steps)
    if cpu is not None:
        progress("cpu baseline: %.3g particle-updates/s on one core, %.3g on %d"
                 % (cpu["value"], cpu["all_cores"]["value"], cpu["all_cores"]["cores"]))

    head = measure(args.workload, args.steps, args.warmup, args.chunk, not args.no_graph,
                   not args.no_tune)
    progress("%s: %.4g particle-updates/s, %.3f ms per step"
             % (args.workload, head["value"], head["ms_per_step"]))
    line = {
        "metric": "particle-updates/s",
        "value": head["value"],
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": head["config"],
        "real_particle_updates_per_s": head["real_particle_updates_per_s"],
        "roofline": head["roofline"],
        "valu_issue": head["valu_issue"],
    }
    for name in [w for w in args.also.split(",") if w]:
        if name not in WORKLOADS:
            raise SystemExit("unknown workload %r" % name)
        steps = 400 if name == "c2" else 100
        sec = measure(name, steps, steps // 10, args.chunk, not args.no_graph, not args.no_tune)
        line[name] = sec
        progress("%s: %.4g particle-updates/s, %.3f ms per step"
                 % (name, sec["value"], sec["ms_per_step"]))
    if args.serve > 0:
        lo, hi = (int(v) for v in args.serve_steps.split(","))
        line["serving"] = serving(args.serve, (lo, hi), int(args.serve_budget * (1 << 30)))
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
