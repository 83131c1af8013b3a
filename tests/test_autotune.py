"""The launch-shape autotuner: its cache keys (CPU) and a tuned solve's
parity with the oracle (GPU)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1808_03801_amd import autotune as A
from paper_1808_03801_amd import problems as P
from tests.parity_util import compare_step


def test_cache_key_separates_what_changes_the_best_shape():
    c = P.cavity_2d(Kn=0.1, n=16, ppc=200)
    assert A.cache_key(c) == "gfx950|dim2|fp32|closed|ppc2^7.5"
    # a band is half an octave of particles per cell
    assert A.cache_key(P.cavity_2d(Kn=0.1, n=16, ppc=210)) == A.cache_key(c)
    assert A.cache_key(P.cavity_2d(Kn=0.1, n=16, ppc=100)) != A.cache_key(c)
    s = P.slit_2d(Kn=0.1, a_cells=3, ppc=100)
    assert "|open|" in A.cache_key(s) and "|dim2|" in A.cache_key(s)
    assert "|fp64|" in A.cache_key(P.couette_1d(ncell=20, ppc=100))
    assert A.cache_key(c, arch="gfx942").startswith("gfx942|")


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["cavity", "slit"])
def test_tuned_choice_is_parity_green(name, tmp_path):
    """the tuner picks among both families; the chosen shape then takes a
    parity-green step against the oracle; a second tuning reads the cache"""
    from paper_1808_03801_amd import usp
    pb = (P.cavity_2d(Kn=0.01, n=16, ppc=80, seed=7) if name == "cavity"
          else P.slit_2d(Kn=0.1, a_cells=3, ppc=40, seed=17))
    ctx = usp.Context(0)
    try:
        g = ctx.add(pb)
        cands = A.candidates(g)
        assert A.W4 in cands and (A.W6 in cands) == (name == "cavity")
        cache = str(tmp_path / "tune.json")
        choice = A.tune(ctx, [g], steps=2, repeats=1, cache=cache)
        assert choice[g.id] in cands and g.shape()[0] == choice[g.id]
        assert A.tune.steps_taken == len(cands) * 3
        again = A.tune(ctx, [g], steps=2, repeats=1, cache=cache)
        assert again == choice and A.tune.steps_taken == 0
        o = O.Oracle(pb)
        o.step(3)
        st = o.get_state()
        g.set_diag(True)
        g.set_state(st)
        o.step(1)
        g.step(1)
        ctx.sync()
        compare_step(pb, o.get_state(), g.get_state(), o.diag(), g.diag(), o.fields(0),
                     g.fields(0))
    finally:
        ctx.close()
