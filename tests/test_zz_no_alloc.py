"""usp_step_noalloc, the step for callers that cannot allocate device
memory, against usp_step: the same instances (four of them, three launch
flavours: 1-D FP32 in the wave shapes, 2-D FP32, 1-D FP64) stepped by each
entry point must reach bit-identical states, over two calls in a row whose
second is smaller (fewer instances and cells, so the static scratch holds
the first call's larger tier lists), and the no-allocation call must not
draw on the device allocator."""
import numpy as np
import pytest

from paper_1808_03801_amd import problems as P


def _problems():
    return [P.couette_1d(Kn=0.00135, ncell=369, ppc=139, precision=32, seed=36),
            P.cavity_2d(Kn=0.01, n=16, ppc=80, seed=7),
            P.sod_1d(ncell=150, mean_ppc=200, seed=6),
            P.couette_1d(ncell=40, ppc=100, seed=3)]


def _same(xa, xb):
    a, b = xa.get_state(), xb.get_state()
    return (np.array_equal(a.counts, b.counts) and np.array_equal(a.parts, b.parts)
            and np.array_equal(a.cells, b.cells, equal_nan=True) and a.step == b.step
            and a.n_samples == b.n_samples)


@pytest.mark.gpu
def test_noalloc_step_matches_usp_step_over_two_calls():
    import torch
    from paper_1808_03801_amd import usp
    ctx = usp.Context(0)
    try:
        pbs = _problems()
        a = [ctx.add(pb) for pb in pbs]  # stepped by usp_step
        b = [ctx.add(pb) for pb in pbs]  # stepped by usp_step_noalloc
        ctx.sync()
        torch.cuda.synchronize()
        n0 = torch.cuda.memory_stats()["allocation.all.allocated"]
        ctx.step_noalloc(b, 6)
        ctx.sync()
        assert torch.cuda.memory_stats()["allocation.all.allocated"] == n0
        ctx.step(a, 6)
        ctx.sync()
        for i, (xa, xb) in enumerate(zip(a, b)):
            assert _same(xa, xb), ("first call", i)
        # second call: a smaller input (the FP32 couette and the FP64 one)
        sub = [0, 3]
        ctx.step_noalloc([b[i] for i in sub], 3)
        ctx.step([a[i] for i in sub], 3)
        ctx.sync()
        for i in range(4):
            assert _same(a[i], b[i]), ("second call", i)
        assert a[0].get_state().step == 9 and a[1].get_state().step == 6
    finally:
        ctx.close()


@pytest.mark.gpu
def test_noalloc_step_refuses_what_its_scratch_cannot_hold():
    from paper_1808_03801_amd import usp
    ctx = usp.Context(0)
    try:
        x = ctx.add(P.couette_1d(ncell=20, ppc=50, seed=1))
        with pytest.raises(usp.UspError) as e:
            ctx.step_noalloc([x] * 1025, 1)  # over 1024 instances
        assert e.value.status == -1
        with pytest.raises(usp.UspError) as e:
            ctx.step_noalloc([x, x], 1)  # listed twice
        assert e.value.status == -1
        ctx.step_noalloc([x], 2)
        ctx.sync()
        assert x.get_state().step == 2
    finally:
        ctx.close()
