"""Pins of P_ne (Eq. 16-18): the gradient-length local Knudsen number on
analytic fields.  Central differences (and one-sided ones at the ends) are
exact for linear fields, so Kn_GLL must equal lambda |dQ/dy| / Q exactly."""
import math

import numpy as np

from oracle import oracle as O
from paper_1808_03801_amd import problems as P


def _moments(S0, U, theta):
    n = len(S0)
    m = np.zeros((n, 13))
    m[:, 0] = S0
    m[:, 1:4] = U
    m[:, 4] = m[:, 5] = m[:, 6] = S0 * theta
    return m


def _lambda(pb, S0, theta):
    """mean free path of a cell from the oracle's own closure (pinned in
    test_oracle_moments by nu tau_c = 0.8): a two-particle set with weight
    sum S0 and temperature theta / R"""
    v = math.sqrt(3.0 * theta)
    parts = np.array([[0, 0, v, 0, 0, S0 / 2], [0, 0, -v, 0, 0, S0 / 2]])
    return O.cell_fields(pb, parts)[1][15]


def test_uniform_field_is_equilibrium():
    pb = P.couette_1d(ncell=8)
    th = pb.gas.R * 273.0
    pne = O.pne_of(pb, _moments(np.full(8, 100.0), np.zeros((8, 3)), th))
    assert np.all(pne == 1.0)


def test_density_gradient():
    pb = P.couette_1d(ncell=10)
    th = pb.gas.R * 273.0
    y = (np.arange(10) + 0.5) * pb.dy
    S0 = 100.0 * (1.0 + 2.0 * y / pb.y1)
    pne = O.pne_of(pb, _moments(S0, np.zeros((10, 3)), th))
    dS0 = 200.0 / pb.y1
    for j in range(10):
        kn = _lambda(pb, S0[j], th) * dS0 / S0[j]
        assert math.isclose(-math.log(pne[j]) * pb.Kn_c, kn, rel_tol=1e-9)


def test_velocity_gradient_uses_sound_speed_below_it():
    pb = P.couette_1d(ncell=10)
    th = pb.gas.R * 273.0
    y = (np.arange(10) + 0.5) * pb.dy
    U = np.zeros((10, 3))
    U[:, 0] = 40.0 * (2 * y / pb.y1 - 1)  # |u| below the sound speed everywhere
    S0 = np.full(10, 100.0)
    pne = O.pne_of(pb, _moments(S0, U, th))
    a = math.sqrt(5.0 / 3.0 * th)
    lam = _lambda(pb, 100.0, th)
    for j in range(10):
        # d|u|/dy: |u| is piecewise linear with a kink at the centre, where the
        # central difference of the two middle cells is zero
        if j in (4, 5):
            continue
        kn = lam * 80.0 / pb.y1 / a
        assert math.isclose(-math.log(pne[j]) * pb.Kn_c, kn, rel_tol=1e-9)


def test_temperature_gradient_2d_magnitude():
    pb = P.cavity_2d(Kn=0.01, n=6)
    R = pb.gas.R
    ix, iy = np.meshgrid(np.arange(6), np.arange(6))
    ix, iy = ix.ravel(), iy.ravel()
    T = 273.0 * (1 + 0.01 * ix + 0.02 * iy)
    S0 = 100.0 * 273.0 / T  # uniform pressure: rho T = const
    pne = O.pne_of(pb, _moments(S0, np.zeros((36, 3)), R * T))
    for c in (7, 14, 21, 0, 35):
        gT = 273.0 * math.hypot(0.01, 0.02) / pb.dx
        kn_T = _lambda(pb, S0[c], R * T[c]) * gT / T[c]
        # density is not linear (1/T); its Kn stays below the temperature one
        assert -math.log(pne[c]) * pb.Kn_c >= kn_T * (1 - 1e-9)
        assert -math.log(pne[c]) * pb.Kn_c < kn_T * 1.1
