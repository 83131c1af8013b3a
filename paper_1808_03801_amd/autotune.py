"""Launch-shape autotuner for the cell kernel.

The cell kernel comes in two families of launch shapes (see usp_set_shape):
workgroup shapes that hold a cell in 256 threads (1, 2, 4, 4|6 and 8
particle slots per thread) and wave shapes that hold a cell in one wave of
64 threads (4 or 6 slots per lane; a CU then keeps four times as many cells
in flight).  An instance's last shape is fixed by its capacity; its first
shape -- and with it the family, the threads per cell and the slots per
thread of the launch that runs most cells -- is a free choice: a small first
shape runs typical cells with fewer registers and less LDS, at the cost of
handing dense cells on to a second launch.  Which is fastest depends on the
cell-count distribution and the instance mix, so it is measured.

Shapes of one family add the same numbers in the same order, so a choice
inside a family never changes results; the two families add in different
orders, so switching family changes the last bits of the moments (every
shape is parity-green against the oracle).  The tuner times the candidates
on the live instances themselves: its trial steps are ordinary steps of the
solves.

Choices can be kept in a JSON cache keyed by the device architecture, the
dimension, the state precision, the boundary set (open faces / the plate or
not) and the band of particles per cell, so that later solves of the same
kind skip the trials.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, List, Optional

W4, W6 = 5, 6  # the wave shapes (64 threads x 4 and x 6 slots)


def _has_open_boundary(pb) -> bool:
    return bool(pb.plate) or any(f.kind == 3 for f in pb.faces)


def candidates(inst) -> List[int]:
    """every first shape the library accepts for this instance: the
    workgroup shapes up to its last, the 4-slot wave shape, and the 6-slot
    wave shape without open faces or the plate"""
    first, last, n = inst.shape()
    out = list(range(last + 1)) + [W4]
    if not _has_open_boundary(inst.pb):
        out.append(W6)
    return out


def ppc_band(pb) -> float:
    """particles per cell of the initial state, in half-octave bands"""
    mean = max(pb.expected_particles() / pb.ncell, 1.0)
    return round(2.0 * math.log2(mean)) / 2.0


def cache_key(pb, arch: str = "gfx950") -> str:
    return "%s|dim%d|fp%d|%s|ppc2^%.1f" % (arch, pb.dim, pb.precision,
                                          "open" if _has_open_boundary(pb) else "closed",
                                          ppc_band(pb))


def _arch() -> str:
    try:
        import torch
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:  # noqa: BLE001 - the architecture is only a cache key
        return "gfx950"


def tune(ctx, instances: List, steps: int = 4, repeats: int = 2,
         cache: Optional[str] = None, verbose: bool = False) -> Dict[int, int]:
    """Picks the first launch shape of every group of `instances` that share
    a cache key and a last shape: each candidate is timed over `steps` steps,
    `repeats` times, with all the instances advancing together as they will
    in production; the fastest per group is kept.  Returns {instance id:
    first shape}.  With `cache`, choices are read from / stored in that JSON
    file under cache_key()."""
    arch = _arch()
    groups: Dict[tuple, list] = {}
    for inst in instances:
        key = (cache_key(inst.pb, arch), inst.shape()[1])
        groups.setdefault(key, []).append(inst)
    known = {}
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            known = json.load(fh)
    choice: Dict[int, int] = {}
    timings = {}
    taken = 0
    for (ckey, last), members in groups.items():
        sig = "%s|last%d" % (ckey, last)
        cands = candidates(members[0])
        if sig in known and int(known[sig]) in cands:
            best = int(known[sig])
        else:
            best, best_t = members[0].shape()[0], float("inf")
            for cand in cands:
                for m in members:
                    m.set_shape(cand)
                ctx.step(instances, 1)  # warm: graph / group set-up outside the timing
                ctx.sync()
                taken += 1
                ts = []
                for _ in range(repeats):
                    t0 = time.perf_counter()
                    ctx.step(instances, steps)
                    ctx.sync()
                    ts.append((time.perf_counter() - t0) / steps)
                    taken += steps
                t = min(ts)
                timings[(sig, cand)] = t
                if verbose:
                    print(f"autotune {sig} first shape {cand}: {t * 1e3:.3f} ms/step", flush=True)
                if t < best_t:
                    best, best_t = cand, t
            known[sig] = best
        for m in members:
            m.set_shape(best)
            choice[m.id] = best
    if cache:
        with open(cache, "w") as fh:
            json.dump(known, fh, indent=1, sort_keys=True)
    tune.last_timings = timings
    tune.steps_taken = taken  # steps every instance advanced while tuning
    return choice
