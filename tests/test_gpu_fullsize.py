"""Parity at the full sizes of the workloads, in the launch configuration the
benchmark times (instances batched in one launch, HIP-graph replay).

The oracle takes a few steps from the initial state, its state is loaded into
the library, and both take one more step; the comparison protocol is the one
of tests/parity_util.py (bit-exact counts, decisions and particle order;
values to the state precision; moments to 1e-5)."""
import numpy as np
import pytest

import bench
from oracle import oracle as O
from paper_1808_03801_amd import problems as P
from tests.parity_util import (compare_step, degenerate_cells, dilate, tie_cells,
                                 value_tie_cells)
from tests.test_gpu_parity import reach


def _oracle_states(pbs, warm):
    out = []
    for pb in pbs:
        o = O.Oracle(pb)
        o.step(warm)
        assert o.error == 0
        out.append(o.get_state())
    return out


def _parity(pbs, warm=2, graph=True, steps=1):
    """steps = 2: one call of two steps, so that the fused relax + move pass
    runs (cells within reach of a tie of the oracle's first step excused)"""
    from paper_1808_03801_amd import usp
    sts = _oracle_states(pbs, warm)
    ctx = usp.Context(0)
    try:
        ctx.set_graph(graph)
        gs = [ctx.add(pb) for pb in pbs]
        for g, st in zip(gs, sts):
            g.set_diag(True)
            g.set_state(st)
        ctx.step(gs, steps)
        ctx.sync()
        for pb, g, st in zip(pbs, gs, sts):
            o = O.Oracle(pb)
            o.set_state(st)
            excuse = excuse_values = None
            if steps == 2:
                o.step(1)
                r = reach(pb, o.get_state())
                # a value tie of the first step changes velocities, and so the
                # second step's flights and counts within reach
                excuse = dilate(pb, tie_cells(o.diag())
                                | value_tie_cells(o.diag(), pb.precision), r)
                excuse_values = dilate(pb, degenerate_cells(o.diag(), o.fields(0))
                                       | value_tie_cells(o.diag(), pb.precision), r)
                o.step(1)
            else:
                o.step(steps)
            rep = {}
            compare_step(pb, o.get_state(), g.get_state(), o.diag(), g.diag(), o.fields(0),
                         g.fields(0), report=rep, excuse=excuse, excuse_values=excuse_values,
                         steps=steps)
            print(pb.name, pb.ncell, "cells", int(st.counts.sum()), "particles", steps,
                  "steps", rep)
    finally:
        ctx.close()


@pytest.mark.gpu
def test_thermal_couette_and_sod_full_size_batched():
    """1000 cells x 500 particles/cell each, FP32, both in every launch"""
    _parity(bench.workload_c2())


@pytest.mark.gpu
def test_thermal_couette_and_sod_full_size_fused_pass():
    """the same pair over two steps in one call: the fused relax + move pass
    that the benchmark times, compared cell by cell and particle by particle"""
    _parity(bench.workload_c2(), steps=2)


@pytest.mark.gpu
@pytest.mark.parametrize("kn", [1e-3, 1e-2, 0.1])
def test_cavity_full_size(kn):
    """128 x 128 cells x 200 particles/cell (3.3 M), FP32"""
    _parity([P.cavity_2d(Kn=kn, seed=21)])


@pytest.mark.gpu
def test_cavity_three_knudsen_full_size_fused_pass():
    """the cavity at Kn = 1e-3, 1e-2 and 0.1 batched in one launch over two
    steps in one call (the fused pass, one-wave cells: the benchmark's
    cavity workload)"""
    _parity(bench.workload_c3(), steps=2)


@pytest.mark.gpu
@pytest.mark.parametrize("kn", [0.01, 0.1])
def test_slit_full_size(kn):
    """400 x 200 cells x 100 particles/cell (8 M), FP32, pressure ratio 2:
    open faces on three sides, the plate, the symmetry plane"""
    _parity([P.slit_2d(Kn=kn, seed=23)])


@pytest.mark.gpu
def test_slit_pair_full_size_fused_pass():
    """the slit at both Knudsen numbers batched, two steps in one call: the
    fused pass of the headline benchmark workload"""
    _parity(bench.workload_c5(), steps=2)


@pytest.mark.gpu
def test_couette_c1_full_size():
    """100 cells x 100 particles/cell, FP64, hard spheres, walls +-100 m/s"""
    _parity([P.couette_1d(seed=0)], warm=5)


def _long_run(pbs, steps):
    from paper_1808_03801_amd import usp
    ctx = usp.Context(0)
    try:
        ctx.set_graph(True)
        gs = [ctx.add(pb) for pb in pbs]
        n0 = [g.num_particles() for g in gs]
        left = steps
        while left > 0:
            k = min(100, left)
            ctx.step(gs, k)
            left -= k
        ctx.sync()
        for pb, g, n in zip(pbs, gs, n0):
            assert g.status() == 0, (pb.name, g.status())
            f = g.fields(0)
            assert np.all(np.isfinite(f)), pb.name
            ratio = g.num_particles() / n
            T = f[:, 5]
            print(pb.name, steps, "steps: particles x%.3f, T %.1f..%.1f K" % (ratio, T.min(), T.max()))
            assert 0.5 < ratio < 2.0
            assert T.min() > 50.0 and T.max() < 2000.0
    finally:
        ctx.close()


@pytest.mark.gpu
@pytest.mark.parametrize("which", ["c1", "c2", "c3", "c5"])
def test_workloads_stay_healthy_over_long_runs(which):
    """every configuration at full size for thousands of steps: no capacity
    or window error, finite fields, particle count and temperatures in range"""
    if which == "c1":
        _long_run([P.couette_1d(seed=0)], 1000)
    elif which == "c2":
        _long_run(bench.workload_c2(), 5000)
    elif which == "c3":
        _long_run([P.cavity_2d(Kn=kn, seed=31) for kn in (1e-3, 1e-2, 0.1)], 2000)
    else:
        _long_run([P.slit_2d(Kn=kn, seed=32) for kn in (0.01, 0.1)], 3000)
