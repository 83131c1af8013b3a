"""Pins of the mean ES target (es_mode ES_MEAN, a variant of step 6): each
reassigned particle takes f_G with alpha replaced by its expectation over the
time distribution of Eq. 29-30 instead of alpha(t) at its own time sample.

What fixes it, independently of the code:
  * the expectation itself: E[e^{-nu t}] over t drawn by Eq. 30 (the
    oracle's time sampler, pinned against its distribution elsewhere),
    computed here by quadrature over the uniform u, equals the closed form
    Pr/(Pr - 1) (e^{(Pr - 1) nu dt} - 1)/(e^{Pr nu dt} - 1);
  * the step's expected stress is linear in alpha, so a homogeneous gas
    relaxes at exactly the rates of the sampled scheme (the closed forms of
    test_oracle_relax).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1808_03801_amd import problems as P
from tests.test_oracle_relax import _aniso_state, _rates


@pytest.mark.parametrize("x", [0.1, 1.0, 4.0, 12.0])
def test_alpha_mean_is_the_expectation_over_the_time_sampler(x):
    Pr = 2.0 / 3.0
    nu, dt = 1.0, x  # nu dt = x
    nues = Pr * nu
    u = (np.arange(200000) + 0.5) / 200000
    t = np.array([O.time_sample(ui, nues * dt, nues, dt) for ui in u[::50]])
    mc = np.mean(np.exp(-nu * t))
    closed = Pr / (Pr - 1.0) * math.expm1((Pr - 1.0) * x) / math.expm1(Pr * x)
    assert abs(mc - closed) < 2e-4 * max(1.0, closed), (mc, closed)


@pytest.mark.parametrize("nu_dt,pne", [(1.0, 0.0), (4.0, 1.0), (1.0, 0.4)])
def test_es_mean_relaxes_at_the_sampled_rates(nu_dt, pne):
    ppc = 1200
    pb = P.homogeneous_box(ncell=500, ppc=ppc, nu_dt=nu_dt, pne=pne, precision=64, seed=3)
    pb = pb.replace(es_mode=P.ES_MEAN)
    o = O.Oracle(pb)
    o.set_state(_aniso_state(pb, ppc))
    f0 = o.fields(0)
    o.step(1)
    assert o.error == 0
    f1 = o.fields(0)
    x = _rates(pb, f0)
    Pr = pb.gas.Pr
    a, b = x * pne / 2, Pr * x * pne / 2
    Rs = (1 - a) / (1 + a) * (pne + (1 - pne) * np.exp(-x))
    Rq = (1 - b) / (1 + b) * (pne + (1 - pne) * np.exp(-Pr * x))
    for s0, s1, R, name in [(f0[:, 10], f1[:, 10], Rs, "sigma_xy"),
                            ((f0[:, 7] - f0[:, 8]) / 2, (f1[:, 7] - f1[:, 8]) / 2, Rs, "xx-yy"),
                            (f0[:, 14], f1[:, 14], Rq, "q_y")]:
        d = s1 - R * s0
        se = d.std() / math.sqrt(len(d))
        assert abs(d.mean()) < 4.5 * se, (name, s1.mean() / s0.mean(), R.mean())


def test_es_mean_needs_pr_other_than_one():
    pb = P.homogeneous_box(ncell=4, ppc=50, precision=64).replace(es_mode=P.ES_MEAN)
    gas = pb.gas
    bad = P.Gas(m=gas.m, kB=gas.kB, mu_ref=gas.mu_ref, T_ref=gas.T_ref, omega=gas.omega, Pr=1.0)
    with pytest.raises(Exception):
        O.Oracle(pb.replace(gas=bad))
