"""A state's steps depend on its inputs only, never on what an earlier user
left in the memory the library is given.

The library allocates through PyTorch's caching allocator, which hands out
recycled blocks with their old contents.  Before each run the small-block
pool (the one the per-cell buffers of these instances come from) is filled
with a value and released, then the same problem is created and stepped in
one long call (fused passes).  The states must agree bit for bit whatever
the value: large leftovers used to reach the hand-on estimate of the pass
that takes a new state's moments, moving cells to a shape that adds in
another order."""
import numpy as np
import pytest

from paper_1808_03801_amd import problems as P

FILLS = (0.0, 2.26e6, float("nan"), 1.0e300)


def _run(ctx, pb, steps, fill, first=None):
    import torch
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if fill is not None:
        # 512 KiB blocks come from the small pool, as the instance's buffers do
        junk = [torch.full((1 << 16,), fill, dtype=torch.float64, device="cuda")
                for _ in range(160)]
        torch.cuda.synchronize()
        del junk
    x = ctx.add(pb)
    if first is not None:
        x.set_shape(first)
    ctx.step([x], steps)
    ctx.sync()
    st = x.get_state()
    x.free()
    return st


def _same(a, b):
    return (np.array_equal(a.counts, b.counts) and np.array_equal(a.parts, b.parts)
            and np.array_equal(a.cells, b.cells, equal_nan=True) and a.step == b.step)


CASES = {
    "couette_fp32_wave": (lambda: P.couette_1d(Kn=0.00135, ncell=369, ppc=139, precision=32,
                                               seed=36), 120, None),
    "couette_fp32_workgroup": (lambda: P.couette_1d(Kn=0.00135, ncell=369, ppc=139,
                                                    precision=32, seed=36), 120, 1),
    "sod_fp32": (lambda: P.sod_1d(ncell=304, mean_ppc=98, seed=53), 120, None),
}


@pytest.mark.gpu
@pytest.mark.parametrize("name", sorted(CASES))
def test_recycled_memory_does_not_change_results(name):
    from paper_1808_03801_amd import usp
    make, steps, first = CASES[name]
    pb = make()
    ctx = usp.Context(0)
    try:
        ref = _run(ctx, pb, steps, None, first)
        for fill in FILLS:
            st = _run(ctx, pb, steps, fill, first)
            assert _same(ref, st), (name, fill)
    finally:
        ctx.close()
