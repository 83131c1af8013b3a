"""Pins of step 6 with the linear map of Eq. 10-11 (es_sampler LINEAR).

The reassigned particles take c = u + sqrt(theta) S z with S = I - k a
sigma / p, k = (1 - Pr) / (2 Pr), a = alpha of Eq. 32 at the particle's time
sample, in place of the Cholesky factor of the target covariance lambda =
theta I + (1 - 1/Pr) alpha sigma / rho.  What fixes its outcome, independently
of the code:

  * S S^T = I - 2 k a sigma/p + k^2 a^2 (sigma/p)^2 and -2 k = 1 - 1/Pr: to
    first order in sigma / p the covariance is lambda, so a weakly
    anisotropic gas relaxes at the closed-form rates of test_oracle_relax;
  * the second order is what separates it from the exact covariance: a
    reassigned particle's second moments exceed those of a Cholesky draw by
    theta k^2 a^2 (sigma/p)^2.  Both samplers turn the same Gaussian draw
    into the velocity and select the same particles, so with P_ne = 0 and no
    conservation correction, after one step from one state, the temperature
    of a cell exceeds the Cholesky run's by T f k^2 E[a^2] tr((sigma/p)^2) / 3
    and its stress by p f k^2 E[a^2] times the trace-free part of
    (sigma/p)^2, f the reassigned fraction and, with a = exp(-nu t) and t
    from the density nu_ES e^{nu_ES t} / (e^{x} - 1) on [0, dt] (Eq. 30,
    x = nu_ES dt = Pr nu dt),
      E[a^2] = Pr (e^{(Pr - 2) nu dt} - 1) / ((Pr - 2) (e^{Pr nu dt} - 1)).
    A map with alpha left out (a = 1) or k's sign turned gives another
    first- or second-order offset.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1808_03801_amd import problems as P
from tests.test_oracle_relax import _aniso_state
from tests.test_oracle_sp import _weak_aniso_state


@pytest.mark.parametrize("pne", [0.0, 0.4, 1.0])
def test_linear_sampler_relaxes_at_the_closed_form_rates(pne):
    ppc = 1200
    pb = P.homogeneous_box(ncell=1600, ppc=ppc, nu_dt=1.0, pne=pne, precision=64, seed=3)
    pb = pb.replace(es_sampler=P.ES_LINEAR)
    o = O.Oracle(pb)
    o.set_state(_weak_aniso_state(pb, ppc))
    f0 = o.fields(0)
    o.step(1)
    assert o.error == 0
    f1 = o.fields(0)
    mu = pb.gas.mu_ref * (f0[:, 5] / pb.gas.T_ref) ** pb.gas.omega
    x = f0[:, 6] / mu * pb.dt
    Pr = pb.gas.Pr
    a, b = x * pne / 2, Pr * x * pne / 2
    Rs = (1 - a) / (1 + a) * (pne + (1 - pne) * np.exp(-x))
    Rq = (1 - b) / (1 + b) * (pne + (1 - pne) * np.exp(-Pr * x))
    for s0, s1, R, name in ((f0[:, 10], f1[:, 10], Rs, "sigma_xy"),
                            ((f0[:, 7] - f0[:, 8]) / 2, (f1[:, 7] - f1[:, 8]) / 2, Rs,
                             "sigma_xx-yy"),
                            (f0[:, 14], f1[:, 14], Rq, "q_y")):
        d = s1 - R * s0
        se = d.std() / math.sqrt(len(d))
        assert abs(d.mean()) < 4.5 * se, (name, s1.mean() / s0.mean(), R.mean())


def test_linear_sampler_second_order_against_cholesky():
    ppc, ncell = 400, 2000
    pb = P.homogeneous_box(ncell=ncell, ppc=ppc, nu_dt=1.0, pne=0.0, precision=64, seed=9)
    pb = pb.replace(conserve_mode=P.CONSERVE_NONE)
    Pr = pb.gas.Pr
    st = _aniso_state(pb, ppc, seed=4)
    runs = {}
    for sampler in (P.ES_CHOLESKY, P.ES_LINEAR):
        o = O.Oracle(pb.replace(es_sampler=sampler))
        o.set_state(st)
        f0 = o.fields(0)
        o.step(1)
        assert o.error == 0
        runs[sampler] = (f0, o.fields(0), o.diag())
    f0, f1c, dc = runs[P.ES_CHOLESKY]
    _, f1l, dl = runs[P.ES_LINEAR]
    # the same particles are reassigned in both runs (the selection does not
    # depend on the sampler)
    assert np.array_equal(dc[:, O.DIAG["n_usp"]], dl[:, O.DIAG["n_usp"]])
    f = dl[:, O.DIAG["n_usp"]] / dl[:, O.DIAG["n_in"]]
    # sigma / p of each cell (xx, yy, zz, xy, xz, yz of the field record)
    p = f0[:, 6]
    M = np.zeros((ncell, 3, 3))
    comps = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
    for c, (i, j) in enumerate(comps):
        M[:, i, j] = M[:, j, i] = f0[:, 7 + c] / p
    M2 = M @ M
    tr2 = np.trace(M2, axis1=1, axis2=2)
    mu = pb.gas.mu_ref * (f0[:, 5] / pb.gas.T_ref) ** pb.gas.omega
    y = f0[:, 6] / mu * pb.dt  # nu dt
    Ea2 = Pr * np.expm1((Pr - 2.0) * y) / ((Pr - 2.0) * np.expm1(Pr * y))
    k = (1.0 - Pr) / (2.0 * Pr)
    w = f * k * k * Ea2
    checks = [("T", (f1l[:, 5] - f1c[:, 5]) / f1c[:, 5], w * tr2 / 3.0)]
    for c, (i, j) in enumerate(comps):
        want = w * (M2[:, i, j] - (tr2 / 3.0 if i == j else 0.0))
        checks.append(("sigma_%d%d" % (i, j), (f1l[:, 7 + c] - f1c[:, 7 + c]) / p, want))
    for name, got, want in checks:
        d = got - want
        se = d.std() / math.sqrt(len(d))
        print("%-9s excess %.3e (predicted %.3e), se %.1e"
              % (name, got.mean(), want.mean(), se))
        if name in ("T", "sigma_00", "sigma_22", "sigma_01"):
            assert abs(want.mean()) > 10.0 * se  # the effect is resolved
        assert abs(d.mean()) < 4.5 * se, name
