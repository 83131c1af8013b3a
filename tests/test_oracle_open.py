"""Pins of the open faces (reservoirs) and of the internal plate (Table 2
step 3 for the Sod tube's open ends and the slit of Section 4.5).

An open face borders a reservoir of gas at rest (number density n,
temperature T).  What kinetic theory fixes, independently of the code:
  * the one-sided number flux of a Maxwellian gas at rest through a plane is
    n sqrt(theta / (2 pi)), theta = k T / m (the effusion rate);
  * the velocities of the molecules crossing the plane follow the
    flux-weighted half-range Maxwellian: normal speed with density
    (v / theta) exp(-v^2 / (2 theta)), so <v_n> = sqrt(pi theta / 2) and
    <v_n^2> = 2 theta; tangential components Maxwellian (mean = the
    reservoir's tangential velocity, variance theta);
  * molecules cross at uniformly distributed times, so the depth reached by
    the end of the step, d = v_n (dt - t_cross), has <d / v_n> = dt / 2;
  * free-molecular effusion from a reservoir into vacuum through a 1-D
    channel: the gas in the channel is the half-range Maxwellian of the
    reservoir, density n / 2, mean velocity sqrt(2 theta / pi), temperature
    theta (3 - 2 / pi) / 3 (normal variance theta (1 - 2 / pi));
  * a channel between two reservoirs in the same state stays in that state.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1808_03801_amd import problems as P


def _p6(c, y, x=0.0):
    return np.array([x, y, c[0], c[1], c[2], 1.0])


def test_open_faces_absorb_leaving_particles():
    pb = P.open_channel_1d(Kn=0.1, ncell=10, ppc=50)
    H = pb.y1
    d, _ = O.advect(pb, _p6([0.0, 1e6, 0.0], 0.999 * H), 9, 0, 0)
    assert d == -1
    d, _ = O.advect(pb, _p6([0.0, -1e6, 0.0], 0.001 * H), 0, 0, 0)
    assert d == -1
    # one that stays inside is untouched by the open faces
    d, r = O.advect(pb, _p6([3.0, 10.0, -2.0], 0.5 * H), 5, 0, 0)
    assert d == 5 and abs(r[1] - (0.5 * H + 10.0 * pb.dt)) <= 1e-15 * H and r[3] == 10.0


def _injected(pb, cell, face, steps):
    out = [O.inject(pb, s, cell, face) for s in range(steps)]
    return [len(x) for x in out], np.concatenate(out)


@pytest.mark.parametrize("face", [2, 3])
def test_entering_particles_follow_the_effusion_flux(face):
    pb = P.open_channel_1d(Kn=0.1, ncell=10, ppc=50, T_lo=300.0, T_hi=300.0, n_hi=0.7)
    cell = 0 if face == 2 else pb.ny - 1
    fc = pb.faces[face]
    th = pb.gas.kB * fc.T / pb.gas.m
    counts, x = _injected(pb, cell, face, 3000)
    rate = fc.n * math.sqrt(th / (2.0 * math.pi)) * pb.dt / pb.Np  # per step, unit area
    # stochastic rounding: every count is floor or ceil of the rate
    assert set(counts) <= {math.floor(rate), math.ceil(rate)}
    assert abs(np.mean(counts) - rate) < 4.0 * 0.5 / math.sqrt(len(counts))
    sgn = 1.0 if face == 2 else -1.0
    vn = sgn * x[:, 3]
    assert np.all(vn > 0.0) and np.all(x[:, 5] == 1.0)
    n = len(vn)
    assert abs(vn.mean() / math.sqrt(math.pi * th / 2.0) - 1.0) < 4.0 * 0.52 / math.sqrt(n)
    assert abs((vn ** 2).mean() / (2.0 * th) - 1.0) < 4.0 * 1.0 / math.sqrt(n)
    for k in (2, 4):
        assert abs(x[:, k].mean()) < 4.0 * math.sqrt(th / n)
        assert abs(x[:, k].var() / th - 1.0) < 4.0 * math.sqrt(2.0 / n)
    # depth reached: uniform crossing times
    y_face = pb.y0 if face == 2 else pb.y1
    depth = np.abs(x[:, 1] - y_face)
    assert abs((depth / vn).mean() / (pb.dt / 2.0) - 1.0) < 4.0 / math.sqrt(3.0 * n)
    assert np.all(depth <= vn * pb.dt)


def test_effusion_into_vacuum_is_the_half_range_maxwellian():
    """free-molecular channel (Kn = 100, relaxation negligible) from an empty
    start; the first quarter of the channel (where every speed class has
    arrived) against the closed forms"""
    pb = P.open_channel_1d(Kn=100.0, ncell=20, ppc=100, n_hi=0.0, empty=True, seed=3)
    o = O.Oracle(pb)
    o.step(1500)
    acc = np.zeros((pb.ncell, 18))
    K = 1500
    for _ in range(K):
        o.step(1)
        acc += o.fields(0)
    assert o.error == 0
    f = acc[:5] / K
    th = pb.gas.kB * 273.0 / pb.gas.m
    n0 = pb.meta["n0"]
    assert np.all(np.abs(f[:, 1] / (pb.gas.m * n0 / 2.0) - 1.0) < 0.025), f[:, 1]
    assert np.all(np.abs(f[:, 3] / math.sqrt(2.0 * th / math.pi) - 1.0) < 0.025), f[:, 3]
    # centred second moments of N particles estimate (1 - 1/N) of the variance
    bias = 1.0 - 1.0 / f[:, 17]
    T_ref = 273.0 * (3.0 - 2.0 / math.pi) / 3.0 * bias
    assert np.all(np.abs(f[:, 5] / T_ref - 1.0) < 0.02), f[:, 5]
    # no particle ever moves towards the source in a collisionless channel:
    # the normal stress is the half-range variance theta (1 - 2/pi)
    p_yy = f[:, 6] + f[:, 8]
    assert np.all(np.abs(p_yy / (f[:, 1] * th * (1.0 - 2.0 / math.pi) * bias) - 1.0) < 0.05)


def test_channel_between_equal_reservoirs_stays_in_their_state():
    """collisional channel (Kn = 0.01, nu dt ~ 1.2), the SP-ESBGK limit
    (P_ne = 0, where equilibrium is exact); count per cell n V / N_p = 200 and
    the temperature estimator's expected (1 - 1/N) T"""
    pb = P.open_channel_1d(Kn=0.01, ncell=20, ppc=200, n_hi=1.0, seed=5).replace(
        pne_mode=P.PNE_FIXED, pne_fixed=0.0)
    o = O.Oracle(pb)
    o.step(200)
    acc = np.zeros((pb.ncell, 18))
    K = 1500
    for _ in range(K):
        o.step(1)
        acc += o.fields(0)
    assert o.error == 0
    f = acc / K
    assert abs(f[:, 17].mean() / 200.0 - 1.0) < 0.02
    assert abs(f[:, 5].mean() / (273.0 * (1.0 - 1.0 / 200.0)) - 1.0) < 0.01
    assert np.all(np.abs(f[:, 3]) < 10.0)


def _slit():
    return P.slit_2d(Kn=0.1, a_cells=2, ppc=20, precision=64)


def test_plate_reflects_and_the_opening_passes():
    pb = _slit()
    a, d = pb.meta["a"], pb.dx
    ix0 = pb.nx // 2  # first column right of the plate
    # towards the plate from the left, at a height it covers
    y = 3.0 * a
    iy = int((y - pb.y0) / pb.dy)
    v = 0.6 * d / pb.dt
    x0 = -0.5 * d
    src = iy * pb.nx + ix0 - 1
    dd, r = O.advect(pb, _p6([v, 0.0, 0.0], y, x0), src, 0, 4)
    assert dd >= 0 and r[0] < 0.0 and r[2] < 0.0 and dd % pb.nx < ix0
    # the same through the opening (below a/2): straight through
    y = 0.2 * a
    iy = int((y - pb.y0) / pb.dy)
    dd, r = O.advect(pb, _p6([v, 0.0, 0.0], y, x0), iy * pb.nx + ix0 - 1, 0, 4)
    assert r[0] > 0.0 and r[2] == v and dd == iy * pb.nx + ix0
    # from the right side too
    dd, r = O.advect(pb, _p6([-v, 0.0, 0.0], 3.0 * a, 0.5 * d), src + 1, 0, 4)
    assert r[0] > 0.0 and r[2] > 0.0


def test_plate_reemits_with_full_accommodation():
    pb = _slit()
    a, d = pb.meta["a"], pb.dx
    th = pb.gas.kB * pb.plate_T / pb.gas.m
    v = 0.6 * d / pb.dt
    vn, vt = [], []
    for s in range(3000):
        # hits the plate half way through the step, then flies off
        dd, r = O.advect(pb, _p6([v, 0.0, 0.0], 4.0 * a, -0.3 * d), 0, s, 7)
        vn.append(-r[2])
        vt.append(r[3])
    vn, vt = np.array(vn), np.array(vt)
    n = len(vn)
    assert np.all(vn > 0.0)
    assert abs(vn.mean() / math.sqrt(math.pi * th / 2.0) - 1.0) < 4.0 * 0.52 / math.sqrt(n)
    assert abs(vt.var() / th - 1.0) < 4.0 * math.sqrt(2.0 / n)


def test_split_open_face_takes_each_chamber_state():
    """the top face of the slit domain borders the upstream reservoir left of
    the plate and the downstream one right of it"""
    pb = _slit()
    top = (pb.ny - 1) * pb.nx
    left, right = top + 2, top + pb.nx - 3
    cl, _ = _injected(pb, left, 3, 2000)
    cr, _ = _injected(pb, right, 3, 2000)
    ratio = np.mean(cl) / np.mean(cr)
    assert abs(ratio / (pb.faces[3].n / pb.faces[3].n_b) - 1.0) < 0.02
    # and the cells in between get nothing through the bottom (specular) face
    assert len(O.inject(pb, 0, 2, 2)) == 0


def test_full_height_plate_is_a_wall():
    """a plate over the whole height separates the chambers: nothing reaches
    the downstream side from an empty start with a vacuum there"""
    pb = P.slit_2d(Kn=0.1, a_cells=2, ppc=20, precision=64, p_ratio=math.inf)
    pb = pb.replace(plate_ylo=pb.y0)
    o = O.Oracle(pb)
    o.step(60)
    st = o.get_state()
    cnt = st.counts.reshape(pb.ny, pb.nx)
    assert cnt[:, : pb.nx // 2].sum() > 0
    assert cnt[:, pb.nx // 2:].sum() == 0


def test_bad_open_configurations_are_refused():
    pb = P.open_channel_1d(Kn=0.1, ncell=10, ppc=50)
    with pytest.raises(Exception):
        O.Oracle(pb.replace(accel=(1.0, 0.0, 0.0)))
    bad = list(pb.faces)
    bad[2] = P.Face(P.BC_OPEN, 273.0, (0.0, 5.0, 0.0), n=1e20)
    with pytest.raises(Exception):
        O.Oracle(pb.replace(faces=bad))
    with pytest.raises(Exception):
        O.Oracle(pb.replace(plate=1, plate_x=0.5, plate_ylo=0.0, plate_yhi=1.0))
