"""Pin of step 5 with Eq. 9's count as printed (select_mode COUNT).

Eq. 9 gives the number of particles of a cell that relax in a step, N_s =
nearest integer of N_c (1 - exp(-nu_ES dt)), nu_ES = Pr nu; the default
reading draws a Bernoulli trial per particle at that rate instead.  What the
count fixes, independently of the code, for a homogeneous gas with P_ne = 0
(no added particles, so Eq. 28 keeps all N_s and deletes none) and without
the conservation correction:

  * every cell reassigns exactly N_s particles;
  * the reassigned particles come from f_G(t), a Gaussian: they carry no
    heat flux, and their stress is the fraction g of sigma that makes the
    Bernoulli scheme relax exactly, (1 - p) + p g = exp(-nu dt) with
    p = 1 - exp(-nu_ES dt) (the closed form pinned in test_oracle_relax);
  * so with f = N_s / N_c one step takes q to (1 - f) q and sigma to
    (1 - f (1 - g)) sigma -- not to exp(-nu_ES dt) q and exp(-nu dt) sigma.

The counts are checked exactly on cells of about 10 particles (N_c p near
1.45: one particle where a Bernoulli draw would spread the count over
0..N_c).  The rates are checked for consistency on cells of 400 particles,
where the moments' sample-mean bias (of order 1 / N_c) is below the
statistical error; there the count and the Bernoulli rate are too close to
tell apart (f = 0.005 against p = 0.0061: 0.3 standard errors over 60 000
cells), so the count itself is what pins the mode.
"""
import math

import numpy as np

from oracle import oracle as O
from paper_1808_03801_amd import problems as P
from tests.test_oracle_relax import _aniso_state


def _count_box(ppc, ncell, nsp, seed):
    """homogeneous anisotropic gas, P_ne = 0, count selection, no
    conservation correction (with one to three particles reassigned per
    cell its shift to the cell's momentum would take their sample mean out
    of their stress); nu dt set so that N_c (1 - exp(-nu_ES dt)) = nsp at
    the mean state"""
    Pr = 2.0 / 3.0
    nu_dt = -math.log(1.0 - nsp / ppc) / Pr
    pb = P.homogeneous_box(ncell=ncell, ppc=ppc, nu_dt=nu_dt, pne=0.0, precision=64, seed=seed)
    assert abs(pb.gas.Pr - Pr) < 1e-15
    pb = pb.replace(select_mode=P.SELECT_COUNT, conserve_mode=P.CONSERVE_NONE)
    o = O.Oracle(pb)
    o.set_state(_aniso_state(pb, ppc, seed=seed + 1))
    f0 = o.fields(0)
    o.step(1)
    assert o.error == 0
    return pb, f0, o.fields(0), o.diag()


def test_count_selection_reassigns_the_eq9_count():
    pb, f0, f1, d = _count_box(10, 20000, 1.45, 7)
    # the selection probability of each cell's f-tilde^* (after the
    # advection of the step; its own rate is pinned in test_oracle_relax)
    p = d[:, O.DIAG["p_sel"]]
    ok = p > 0.0  # a cell of fewer than two particles does not relax
    assert ok.mean() > 0.99
    n_in = d[ok, O.DIAG["n_in"]]
    ns = np.floor(n_in * p[ok] + 0.5)
    # Eq. 9 in every cell (a product within rounding of a half integer may go
    # either way)
    sel = d[ok, O.DIAG["n_sel"]]
    assert np.mean(sel == ns) > 0.99
    assert np.all(np.abs(sel - ns) <= 1)
    assert np.all(d[ok, O.DIAG["n_usp"]] == sel)
    assert np.all(d[:, O.DIAG["n_del"]] == 0)
    assert np.all(d[:, O.DIAG["n4"]] == 0) and np.all(d[:, O.DIAG["n7"]] == 0)
    # a Bernoulli draw would spread the count of a cell over 0..N_c: here it
    # is the rounded product in every cell, so for cells of one size and
    # nearly one rate it is one number
    same = (n_in == 10) & (np.abs(n_in * p[ok] - 1.45) < 0.03)
    assert same.sum() > 200 and np.all(sel[same] == 1)


def test_count_selection_relaxes_at_the_rate_of_its_count():
    """consistency of the reassigned fraction with the relaxation: heat flux
    and stress decay as 1 - f and 1 - f (1 - g) (cells of 400 particles,
    where the moments' sample-mean bias is below the statistical error; the
    count and the Bernoulli rate differ here by less than that error, so
    this checks the resampling of the count's particles, not the count)"""
    Pr = 2.0 / 3.0
    pb, f0, f1, d = _count_box(400, 20000, 2.45, 11)
    p = d[:, O.DIAG["p_sel"]]
    x = -np.log1p(-p) / Pr  # nu dt of each cell's f-tilde^*
    f = d[:, O.DIAG["n_sel"]] / d[:, O.DIAG["n_in"]]
    g = (np.exp(-x) - (1.0 - p)) / p
    Rs, Rq = 1.0 - f * (1.0 - g), 1.0 - f
    for s0, s1, R, name in ((f0[:, 10], f1[:, 10], Rs, "sigma_xy"),
                            (f0[:, 14], f1[:, 14], Rq, "q_y")):
        dd = s1 - R * s0
        se = dd.std() / math.sqrt(len(dd))
        assert abs(dd.mean()) < 4.5 * se, (name, (s1.mean() / s0.mean()), R.mean())


def test_bernoulli_default_is_unchanged_by_the_flag():
    """select_mode BERNOULLI (the default) leaves the state as before the
    flag existed: the same step with the flag spelled out gives the same
    state bit for bit"""
    pb = P.homogeneous_box(ncell=50, ppc=200, nu_dt=1.0, pne=1.0, precision=64, seed=3)
    a, b = O.Oracle(pb), O.Oracle(pb.replace(select_mode=P.SELECT_BERNOULLI))
    a.step(3)
    b.step(3)
    sa, sb = a.get_state(), b.get_state()
    assert np.array_equal(sa.parts, sb.parts) and np.array_equal(sa.cells, sb.cells)
