"""Pins of the GLL switch's velocity term (Eq. 16-18): lambda |grad |u|| over
max(|u|, sqrt(5 theta / 3)) (the convention of the criterion's authors,
gll_u = 0) or over |u| as printed (gll_u = 1).

What the definitions fix, independently of the code:
  * where every cell moves faster than sound the two agree exactly;
  * elsewhere the printed form gives the larger Knudsen number, so P_ne can
    only drop;
  * a cell at rest inside a velocity gradient is fully rarefied under the
    printed form: P_ne = 0.
"""
import numpy as np

from oracle import oracle as O
from paper_1808_03801_amd import problems as P


def _shear(u0, ncell=40, seed=3):
    """Couette-like layer with a linear velocity u0 + (y - H/2) * 200 / H,
    uniform density and temperature, P_ne from the instantaneous fields"""
    pb = P.couette_1d(Kn=0.05, ncell=ncell, ppc=400, precision=64, seed=seed)
    H = pb.meta["H"]
    y = (np.arange(ncell) + 0.5) * H / ncell
    iu = np.zeros((ncell, 3))
    iu[:, 0] = u0 + (y - 0.5 * H) * 200.0 / H
    return pb.replace(init_u=iu, pne_mode=P.PNE_GLL_INST, avg_init=0)


def _pne(pb):
    return O.Oracle(pb).fields(0)[:, 16]


def test_supersonic_layer_gives_the_same_p_ne():
    pb = _shear(2000.0)
    a = _pne(pb)
    b = _pne(pb.replace(gll_u=P.GLL_U_LITERAL))
    assert np.array_equal(a, b)
    assert np.all((a > 0.0) & (a <= 1.0))


def test_printed_form_only_lowers_p_ne_and_zeroes_a_cell_at_rest():
    pb = _shear(0.0)
    a = _pne(pb)
    b = _pne(pb.replace(gll_u=P.GLL_U_LITERAL))
    assert np.all(b <= a)
    assert np.any(b < 0.5 * a)
    # the layer's mid cells move at a few m/s (sampling noise of 400
    # particles, ~12 m/s): |u| is far below lambda |d|u|/dy|, so the printed
    # term drives P_ne towards zero there, where the sound-speed form keeps
    # the layer near-continuum
    mid = slice(pb.ncell // 2 - 2, pb.ncell // 2 + 2)
    assert np.all(b[mid] < 0.05), b[mid]
    assert b[mid].min() < 1e-3
    assert np.all(a[mid] > 0.5), a[mid]
