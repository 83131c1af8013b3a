"""Launch-shape autotuner for the cell kernel.

The cell kernel comes in five shapes (256 threads x 1, 2, 4, 4|6 and 8
particle slots per thread, see usp_set_shape).  An instance's last shape is
fixed by its capacity; its first shape is a free choice: a small first shape
runs typical cells with fewer registers and less LDS, at the cost of handing
dense cells on to a second launch.  Which is fastest depends on the cell
count distribution and the instance mix, so it is measured.

Every shape adds the same numbers in the same order (all use 256 threads,
particle j in thread j mod 256), so the choice never changes results.  The
tuner therefore times the candidates on the live instances themselves: its
trial steps are ordinary steps of the solves.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, List, Optional


def _flavour(inst):
    first, last, n = inst.shape()
    return (inst.pb.precision, inst.pb.dim, last), n


def tune(ctx, instances: List, steps: int = 4, repeats: int = 2,
         cache: Optional[str] = None, verbose: bool = False) -> Dict[int, int]:
    """Picks the first launch shape of every flavour group of `instances`
    (same state precision, dimension and last shape): each candidate (every
    shape up to the group's last) is timed over `steps` steps, `repeats`
    times, with all the instances advancing together as they will in
    production; the fastest per group is kept.  Returns {instance id: first
    shape}.  With `cache`, choices are stored in / read from that JSON file,
    keyed by the flavour and the instance sizes."""
    groups: Dict[tuple, list] = {}
    nshape = 0
    for inst in instances:
        key, nshape = _flavour(inst)
        groups.setdefault(key, []).append(inst)
    known = {}
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            known = json.load(fh)
    choice: Dict[int, int] = {}
    timings = {}
    taken = 0
    for key, members in groups.items():
        sig = json.dumps([list(key), sorted(m.pb.ncell * m.pb.max_ppc for m in members)])
        if sig in known:
            best = int(known[sig])
        else:
            last = key[2]
            best, best_t = last, float("inf")
            for cand in range(last + 1):
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
                timings[(key, cand)] = t
                if verbose:
                    print(f"autotune {key} first shape {cand}: {t * 1e3:.3f} ms/step", flush=True)
                if t < best_t:
                    best, best_t = cand, t
            known[sig] = best
        for m in members:
            m.set_shape(best)
            choice[m.id] = best
    if cache:
        with open(cache, "w") as fh:
            json.dump(known, fh, indent=1)
    tune.last_timings = timings
    tune.steps_taken = taken  # steps every instance advanced while tuning
    return choice
