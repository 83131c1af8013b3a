"""The solve server: request mix (CPU) and continuous batching on the GPU."""
import math

import numpy as np
import pytest

from paper_1808_03801_amd import problems as P
from paper_1808_03801_amd import serve as S


def test_request_trace_mix():
    reqs = S.request_trace(256, seed=0)
    assert len(reqs) == 256
    arr = np.array([r.arrival for r in reqs])
    assert np.all(np.diff(arr) > 0)
    # Poisson at 50/s: mean gap 20 ms (256 samples: within 20 %)
    assert abs(np.diff(arr).mean() - 0.02) < 0.004
    assert {r.kind for r in reqs} == set(S.KINDS)
    kn = np.array([r.Kn for r in reqs])
    assert kn.min() >= 1e-3 and kn.max() <= 1.0
    assert all(50 <= r.ncell <= 400 and 50 <= r.ppc <= 200 and 2000 <= r.steps <= 10000
               for r in reqs)
    assert [r.seed for r in reqs] == list(range(256))
    again = S.request_trace(256, seed=0)
    assert [dataclass_tuple(a) for a in reqs] == [dataclass_tuple(b) for b in again]


def dataclass_tuple(r):
    return (r.kind, r.Kn, r.ncell, r.ppc, r.steps, r.seed, r.arrival)


@pytest.mark.parametrize("kind", S.KINDS)
def test_request_problem(kind):
    r = S.Request(kind, Kn=0.01, ncell=80, ppc=100, steps=10, seed=3)
    pb = S.build_problem(r)
    assert pb.ncell == 80 and pb.precision == 32 and pb.seed == 3
    assert pb.weight_mode == P.WEIGHT_LITERAL
    # dt / tau_c = min(5, 0.3 / (Kn ncell)) = 0.375
    tau = pb.meta.get("tau0", pb.meta.get("tau_l"))
    assert math.isclose(pb.dt / tau, 0.375, rel_tol=1e-12)


def _small_trace(n, rate, seed):
    return S.request_trace(n, rate=rate, steps=(40, 120), cells=(20, 60), ppc=(50, 80),
                           kn=(3e-3, 0.3), seed=seed)


def _run_server(ctx, reqs, budget, chunk=16):
    srv = S.Server(ctx, budget=budget, chunk=chunk)
    futs = [srv.submit(r) for r in reqs]
    srv.run()
    return srv, [f.result() for f in futs]


@pytest.mark.gpu
def test_each_result_same_alone_and_in_the_mix():
    from paper_1808_03801_amd import usp
    reqs = _small_trace(8, rate=2000.0, seed=5)
    ctx = usp.Context(0)
    try:
        srv, mixed = _run_server(ctx, reqs, budget=2 << 30)
        assert srv.max_active >= 4  # arrivals overlap: solves shared launches
        # the host waited only when a solve finished (or every few chunks)
        assert srv.syncs < srv.chunks, (srv.syncs, srv.chunks)
        alone = S.run_plain(ctx, reqs)
        by_seed = {r.request.seed: r for r in alone}
        for m in mixed:
            a = by_seed[m.request.seed]
            assert np.array_equal(m.fields, a.fields), m.request
            assert np.array_equal(m.avg_fields, a.avg_fields), m.request
    finally:
        ctx.close()


@pytest.mark.gpu
def test_admission_by_footprint_queues_and_completes():
    from paper_1808_03801_amd import usp
    reqs = _small_trace(6, rate=5000.0, seed=6)
    fps = [usp.footprint(S.build_problem(r)) for r in reqs]
    budget = int(2.2 * max(fps))
    ctx = usp.Context(0)
    try:
        srv, mixed = _run_server(ctx, reqs, budget=budget)
        assert srv.max_active <= 2
        assert sorted(m.request.seed for m in mixed) == sorted(r.seed for r in reqs)
        alone = {r.request.seed: r for r in S.run_plain(ctx, reqs)}
        for m in mixed:
            assert np.array_equal(m.fields, alone[m.request.seed].fields)
        # a request larger than the whole budget is refused, not queued forever
        big = S.Server(ctx, budget=min(fps) // 2)
        with pytest.raises(MemoryError):
            big.submit(reqs[0]).result()
    finally:
        ctx.close()
