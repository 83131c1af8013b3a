"""Continuous-batching solve server over libusp.

Requests name a 1-D solve (Couette, Poiseuille or Sod tube at a Knudsen
number, cell count, particles per cell and step count).  The server admits
queued requests in arrival order while their HBM footprint (usp_footprint)
fits the budget, keeps every admitted solve's particle state resident, and
advances all active solves together: each chunk of steps is one batched
usp_step call over every active instance, so a request that arrives while
others run joins the next chunk, and its work overlaps theirs in the same
kernel launches.  Finished solves return their moment fields to the host and
free their memory, which admits the next requests.

Each instance's result does not depend on what it was batched with (every
cell is computed by the same code from its own data and its own Philox
streams), so a solve returns the same moments alone and in the mix.

The plain baseline (`run_plain`) runs the same requests one at a time in
arrival order, each on its own.
"""
from __future__ import annotations

import collections
import concurrent.futures
import dataclasses
import math
import time
from typing import Dict, List, Optional

import numpy as np

from . import problems as P

KINDS = ("couette", "poiseuille", "sod")


@dataclasses.dataclass
class Request:
    kind: str          # couette | poiseuille | sod
    Kn: float
    ncell: int
    ppc: int
    steps: int
    seed: int = 0
    arrival: float = 0.0  # seconds after the start of a trace


@dataclasses.dataclass
class Result:
    request: Request
    fields: np.ndarray     # [ncell][18] cell fields of the final state (usp_get_fields)
    avg_fields: np.ndarray  # the same from the Eq. 34 averages
    t_admit: float
    t_done: float

    @property
    def latency(self) -> float:
        return self.t_done - self.request.arrival


def build_problem(req: Request) -> P.Problem:
    """The solve a request names: argon, FP32 state, 1-D,
    dt = min(5 tau_c, 0.3 dx / mean speed), i.e. dt / tau_c = min(5, 0.3 / (Kn ncell)),
    AVG J-moments with the added-batch projection, and the added-particle
    weights of Eq. 26 as printed (they scale with dt, so that at
    nu_ES dt < 1 the weights stay small on cells of 50-200 particles; at
    nu_ES dt >= 1 both weight readings are the same).  Couette plates at
    +-50 m/s; Poiseuille dp/dx = 8 mu U_max / H^2 with U_max = 50 m/s; Sod as
    the paper's tube (density ratio 8, pressure ratio 10) with Kn = lambda_l / L."""
    dto = min(5.0, 0.3 / (req.Kn * req.ncell))
    if req.kind == "couette":
        pb = P.couette_1d(Kn=req.Kn, U_w=50.0, ncell=req.ncell, ppc=req.ppc, dt_over_tau=dto,
                          omega=0.81, precision=32, seed=req.seed)
        pb = pb.replace(jmom_mode=P.JMOM_AVG, spawn_projection=1, avg_init=0)
    elif req.kind == "poiseuille":
        gas = P.Gas(omega=0.81)
        lam0 = P.standard_state(gas, 273.0)[2]
        H = lam0 / req.Kn
        dpdx = 8.0 * gas.mu(273.0) * 50.0 / (H * H)
        pb = P.poiseuille_1d(Kn=req.Kn, dpdx=dpdx, ncell=req.ncell, ppc=req.ppc,
                             dt_over_tau=dto, seed=req.seed)
    elif req.kind == "sod":
        pb = P.sod_1d(Kn=req.Kn, ncell=req.ncell, mean_ppc=req.ppc, dt_over_tau=dto,
                      seed=req.seed)
    else:
        raise ValueError(f"unknown request kind {req.kind!r}")
    return pb.replace(weight_mode=P.WEIGHT_LITERAL)


def request_trace(n: int, rate: float = 50.0, steps=(2000, 10000), cells=(50, 400),
                  ppc=(50, 200), kn=(1e-3, 1.0), seed: int = 0) -> List[Request]:
    """n requests with Poisson arrivals at `rate` per second; kind uniform over
    Couette / Poiseuille / Sod, Kn log-uniform in `kn`, cells, particles per
    cell and steps uniform in their ranges; request i has seed i."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        out.append(Request(kind=KINDS[int(rng.integers(0, 3))],
                           Kn=float(math.exp(rng.uniform(math.log(kn[0]), math.log(kn[1])))),
                           ncell=int(rng.integers(cells[0], cells[1] + 1)),
                           ppc=int(rng.integers(ppc[0], ppc[1] + 1)),
                           steps=int(rng.integers(steps[0], steps[1] + 1)), seed=i, arrival=t))
    return out


class Server:
    """Admits requests by HBM footprint and advances every admitted solve in
    shared batched launches, `chunk` steps at a time."""

    def __init__(self, ctx, budget: int = 2 << 30, chunk: int = 50, graph: bool = True,
                 sync_every: int = 8):
        from . import usp
        self.usp = usp
        self.ctx = ctx
        self.budget = int(budget)
        self.chunk = int(chunk)
        self.graph = bool(graph)
        self.sync_every = int(sync_every)
        self._queue: collections.deque = collections.deque()
        self.max_active = 0
        self.chunks = 0
        self.syncs = 0

    def submit(self, req: Request) -> concurrent.futures.Future:
        fut: concurrent.futures.Future = concurrent.futures.Future()
        pb = build_problem(req)
        fp = self.usp.footprint(pb)
        if fp > self.budget:
            fut.set_exception(MemoryError(f"request needs {fp} B, budget {self.budget} B"))
            return fut
        self._queue.append((req, pb, fp, fut))
        return fut

    def run(self, clock=time.perf_counter, t0: Optional[float] = None) -> None:
        """Serves everything submitted.  Requests become eligible at
        t0 + request.arrival (t0 = now by default); the loop admits eligible
        requests in order while their footprint fits, steps all active solves
        by min(chunk, fewest remaining steps), and retires finished ones.

        The host waits for the device only when a solve has finished (its
        fields are copied out and its memory freed), when nothing is left to
        step, or every `sync_every` chunks (to notice a failed solve early);
        between those the chunks are queued on the stream back to back, and
        with `graph` a chunk over an unchanged set of solves replays the HIP
        graph captured for it.  Admitting a request creates its instance,
        which waits for the stream."""
        t0 = clock() if t0 is None else t0
        self.ctx.set_graph(self.graph)
        active: Dict[int, list] = {}
        used = 0
        queue = collections.deque(sorted(self._queue, key=lambda e: e[0].arrival))
        self._queue.clear()
        pending = 0
        while queue or active:
            now = clock() - t0
            while queue and queue[0][0].arrival <= now and used + queue[0][2] <= self.budget:
                req, pb, fp, fut = queue.popleft()
                inst = self.ctx.add(pb)
                used += fp
                active[inst.id] = [inst, req, req.steps, fut, fp, clock() - t0]
            if not active:
                if queue:
                    time.sleep(max(0.0, queue[0][0].arrival - (clock() - t0)))
                continue
            self.max_active = max(self.max_active, len(active))
            k = min(self.chunk, min(a[2] for a in active.values()))
            self.ctx.step([a[0] for a in active.values()], k)
            self.chunks += 1
            pending += 1
            finished = False
            for a in active.values():
                a[2] -= k
                finished = finished or a[2] == 0
            if not (finished or pending >= self.sync_every):
                continue
            try:
                self.ctx.sync()
            except self.usp.UspError:
                pass  # a solve failed (sticky, its own): found and retired below
            self.syncs += 1
            pending = 0
            done, failed = [], []
            for iid, a in active.items():
                if a[0].status() != 0:
                    failed.append(iid)
                elif a[2] == 0:
                    done.append(iid)
            for iid in failed:
                inst, req, _, fut, fp, _ = active.pop(iid)
                err = self.usp.UspError(inst.status(), "solve failed on the device")
                inst.free()
                used -= fp
                fut.set_exception(err)
            for iid in done:
                inst, req, _, fut, fp, t_admit = active.pop(iid)
                f0, f1 = inst.fields(0), inst.fields(1)
                inst.free()
                used -= fp
                fut.set_result(Result(req, f0, f1, t_admit, clock() - t0))
        self.ctx.set_graph(False)


def run_plain(ctx, reqs: List[Request], clock=time.perf_counter, chunk: int = 1000,
              t0: Optional[float] = None) -> List[Result]:
    """The baseline: one request at a time in arrival order, each alone."""
    t0 = clock() if t0 is None else t0
    out = []
    for req in sorted(reqs, key=lambda r: r.arrival):
        wait = req.arrival - (clock() - t0)
        if wait > 0:
            time.sleep(wait)
        t_admit = clock() - t0
        inst = ctx.add(build_problem(req))
        left = req.steps
        while left > 0:
            k = min(chunk, left)
            ctx.step([inst], k)
            left -= k
        ctx.sync()
        f0, f1 = inst.fields(0), inst.fields(1)
        inst.free()
        out.append(Result(req, f0, f1, t_admit, clock() - t0))
    return out


def summarize(results: List[Result], wall: float) -> dict:
    lat = np.array([r.latency for r in results])
    return {"requests": len(results), "wall_s": wall, "solves_per_s": len(results) / wall,
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean())}
