"""Pins of the oracle's moments (Eq. 1), gas closure (Eq. 35-37) and the
raw-sum bookkeeping used for time averaging (Eq. 34)."""
import math

import numpy as np

from oracle import oracle as O
from paper_1808_03801_amd import problems as P


def _pb(**kw):
    return P.couette_1d(ncell=4, ppc=10, **kw)


def _parts(c, w=None):
    c = np.asarray(c, float)
    n = c.shape[0]
    out = np.zeros((n, 6))
    out[:, 2:5] = c
    out[:, 5] = 1.0 if w is None else w
    return out


def test_two_particle_closed_form():
    # two unit-weight particles at +-v along x: u = 0, p_xx = rho v^2,
    # p = rho v^2 / 3, sigma_xx = 2/3 rho v^2, sigma_yy = sigma_zz = -1/3 rho v^2, q = 0
    pb = _pb()
    v = 300.0
    mom, f = O.cell_fields(pb, _parts([[v, 0, 0], [-v, 0, 0]]))
    F = pb.gas.m * pb.Np / pb.vcell
    rho = 2 * F
    assert f[0] == 1.0
    assert math.isclose(f[1], rho, rel_tol=1e-15)
    assert math.isclose(f[3], rho * v * v / 3, rel_tol=1e-14)
    assert math.isclose(f[2], v * v / 3 / pb.gas.R, rel_tol=1e-14)
    assert np.allclose(f[4:10], [2 / 3 * rho * v * v, -rho * v * v / 3, -rho * v * v / 3, 0, 0, 0],
                       rtol=1e-14, atol=1e-12 * rho * v * v)
    assert np.allclose(f[10:13], 0.0, atol=1e-9)


def test_skewed_three_particles_heat_flux():
    # velocities (a,0,0), (a,0,0), (-2a,0,0): u = 0, C^2 C_x sums to
    # 2 a^3 - 8 a^3 = -6 a^3, so q_x = F * (-6 a^3) / 2
    pb = _pb()
    a = 200.0
    mom, f = O.cell_fields(pb, _parts([[a, 0, 0], [a, 0, 0], [-2 * a, 0, 0]]))
    F = pb.gas.m * pb.Np / pb.vcell
    assert np.allclose(mom[1:4], 0.0, atol=1e-12)
    assert math.isclose(f[10], F * (-6 * a**3) / 2, rel_tol=1e-13)
    assert abs(f[11]) < 1e-9 and abs(f[12]) < 1e-9


def test_galilean_rotation_and_weight_invariance():
    pb = _pb()
    rng = np.random.default_rng(4)
    c = rng.normal(0, 300, (50, 3)) + rng.gamma(2.0, 50, (50, 3))
    w = rng.uniform(0.5, 1.5, 50)
    mom, f = O.cell_fields(pb, _parts(c, w))
    # Galilean shift: u shifts, T, sigma, q unchanged
    V = np.array([120.0, -40.0, 7.0])
    mom2, f2 = O.cell_fields(pb, _parts(c + V, w))
    assert np.allclose(mom2[1:4], mom[1:4] + V, rtol=1e-12, atol=1e-9)
    assert np.allclose(f2[1:13], f[1:13], rtol=1e-9, atol=1e-9 * abs(f[3]))
    # rotation: sigma -> R sigma R^T, q -> R q
    th = 0.7
    Rm = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1.0]])
    mom3, f3 = O.cell_fields(pb, _parts(c @ Rm.T, w))
    s = f[4:10]
    S = np.array([[s[0], s[3], s[4]], [s[3], s[1], s[5]], [s[4], s[5], s[2]]])
    SR = Rm @ S @ Rm.T
    s3 = f3[4:10]
    assert np.allclose([SR[0, 0], SR[1, 1], SR[2, 2], SR[0, 1], SR[0, 2], SR[1, 2]], s3,
                       rtol=1e-9, atol=1e-9 * abs(f[3]))
    assert np.allclose(Rm @ f[10:13], f3[10:13], rtol=1e-9, atol=1e-9 * abs(f[10:13]).max())
    assert math.isclose(f3[2], f[2], rel_tol=1e-12)
    # weight scaling: rho, p, sigma, q scale; T and u do not
    mom4, f4 = O.cell_fields(pb, _parts(c, 3.0 * w))
    assert math.isclose(f4[1], 3 * f[1], rel_tol=1e-14)
    assert math.isclose(f4[2], f[2], rel_tol=1e-12)
    assert np.allclose(f4[4:13], 3 * f[4:13], rtol=1e-12, atol=1e-12 * abs(f[3]))


def test_maxwellian_sample_moments():
    pb = _pb()
    T = 273.0
    th = pb.gas.R * T
    rng = np.random.default_rng(5)
    n = 200000
    c = rng.normal(0, math.sqrt(th), (n, 3))
    mom, f = O.cell_fields(pb, _parts(c))
    assert abs(f[2] / T - 1) < 4 * math.sqrt(2 / (3 * n))
    p = f[3]
    assert np.all(np.abs(f[4:10] / p) < 4 * math.sqrt(2.0 / n) * 2)
    assert np.all(np.abs(f[10:13] / (p * math.sqrt(th))) < 4 * math.sqrt(15.0 / n))


def test_collision_frequency_times_collision_time_is_0_8():
    # nu = p / mu (Eq. 4) and tau_c from Eq. 36-37 give nu tau_c = 16/20 for
    # every state and every viscosity law.
    for omega in (0.5, 0.81):
        pb = _pb(omega=omega)
        rng = np.random.default_rng(6)
        for T in (150.0, 273.0, 900.0):
            c = rng.normal(0, math.sqrt(pb.gas.R * T), (5000, 3))
            mom, f = O.cell_fields(pb, _parts(c))
            nu, tau = f[13], f[16]
            assert math.isclose(nu * tau, 0.8, rel_tol=1e-12)


def test_argon_standard_state_numbers():
    # viscosity law Eq. 35 at T_ref returns mu_ref; lambda and tau_c of
    # argon at 1 atm, 273 K with mu = 2.117e-5 Pa s
    pb = _pb(omega=0.81)
    n0 = P.P_ATM / (P.K_B * 273.0)
    th = pb.gas.R * 273.0
    rng = np.random.default_rng(7)
    c = rng.normal(0, math.sqrt(th), (4000, 3))
    # rescale the sample to exactly T = 273 K so that the closure is evaluated
    # at the standard state
    c -= c.mean(0)
    c *= math.sqrt(3 * th * 4000 / (c**2).sum())
    parts = _parts(c)
    # weights so that rho = m n0
    F = pb.gas.m * pb.Np / pb.vcell
    parts[:, 5] = pb.gas.m * n0 / (F * 4000)
    mom, f = O.cell_fields(pb, parts)
    assert math.isclose(f[14], 2.117e-5, rel_tol=1e-12)
    assert math.isclose(f[15], 6.3596e-8, rel_tol=2e-4)
    assert math.isclose(f[16], 1.6715e-10, rel_tol=2e-4)


def test_first_average_equals_instantaneous_fields():
    # Eq. 34 starts from the first sample; fields derived from averaged raw
    # sums must then equal those from the two-pass centred moments.
    pb = P.couette_1d(ncell=20, ppc=50, U_w=200.0, avg_init=0)
    o = O.Oracle(pb)
    o.step(1)
    a, b = o.fields(0), o.fields(1)
    p = np.abs(a[:, 6]).max()
    assert np.allclose(a[:, 0:5], b[:, 0:5], rtol=1e-10, atol=1e-9)
    assert np.allclose(a[:, 5:16], b[:, 5:16], rtol=1e-7, atol=1e-9 * p)
