"""Pins of Table 2 step 3 (advection, walls, cell index) and of the stable
counting sort by cell."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O
from paper_1808_03801_amd import problems as P


def _one(c, y, x=0.0):
    return np.array([x, y, c[0], c[1], c[2], 1.0])


def test_free_flight_is_one_fma():
    pb = P.couette_1d(ncell=10, precision=32)
    y = np.float32(0.37 * pb.y1)
    cy = np.float32(123.25)
    d, r = O.advect(pb, _one([1.0, float(cy), 0.0], float(y)), 3, 0, 0)
    # float32 fma done exactly in double then rounded once
    expect = np.float32(float(cy) * float(np.float32(pb.dt)) + float(y))
    assert r[1] == float(expect)
    assert d == int(math.floor((r[1] - pb.y0) * pb.inv_dy))


def test_specular_and_periodic_faces():
    pb = P.sod_1d(ncell=10, precision=64)
    H = pb.y1
    cy = -0.3 * H / pb.dt
    y = 0.13 * H
    d, r = O.advect(pb, _one([5.0, cy, 2.0], y), 1, 0, 0)
    # mirror image of the free flight about y = 0
    assert math.isclose(r[1], -(y + cy * pb.dt), rel_tol=1e-12)
    assert r[3] == -cy and r[2] == 5.0 and r[4] == 2.0
    assert d == 1
    # periodic
    pbp = P.homogeneous_box(ncell=10, precision=64)
    H = pbp.y1
    cy = 0.45 * H / pbp.dt
    y = 0.8 * H
    d, r = O.advect(pbp, _one([0.0, cy, 0.0], y), 8, 0, 0)
    assert math.isclose(r[1], y + cy * pbp.dt - H, rel_tol=1e-12)
    assert r[3] == cy and d == int(math.floor(r[1] / pbp.dy))
    # several periods in one step
    cy = 2.3 * H / pbp.dt
    d, r = O.advect(pbp, _one([0.0, cy, 0.0], y), 8, 0, 0)
    assert math.isclose(r[1], (y + cy * pbp.dt) % H, rel_tol=1e-9)


def test_diffuse_wall_reemission_distribution():
    # full accommodation: the re-emitted normal speed has the flux-weighted
    # (Rayleigh) law with scale sqrt(theta_w); tangential components are
    # Maxwellian about the wall velocity; the particle flies the remaining
    # time from the wall.
    Tw = 300.0
    pb = P.couette_1d(ncell=10, precision=64, U_w=80.0)
    pb.faces[2] = P.Face(P.BC_DIFFUSE, Tw, (-80.0, 0.0, 0.0))
    thw = pb.gas.R * Tw
    y0 = 0.02 * pb.y1
    cy = -2.0 * y0 / pb.dt  # hits the wall at dt/2
    n = 6000
    vn, vt, vz, dist = [], [], [], []
    for i in range(n):
        d, r = O.advect(pb, _one([0.0, cy, 0.0], y0), 0, i, 5)
        vn.append(r[3])
        vt.append(r[2])
        vz.append(r[4])
        dist.append(r[1] - (r[3] * pb.dt / 2))
    vn, vt, vz, dist = map(np.array, (vn, vt, vz, dist))
    assert np.all(vn > 0)
    assert stats.kstest(vn, stats.rayleigh(scale=math.sqrt(thw)).cdf).pvalue > 1e-4
    assert stats.kstest((vt + 80.0) / math.sqrt(thw), "norm").pvalue > 1e-4
    assert stats.kstest(vz / math.sqrt(thw), "norm").pvalue > 1e-4
    # remaining flight of dt/2 from the wall (multi-hit traces aside)
    single = vn * pb.dt / 2 < pb.y1
    assert np.allclose(dist[single], 0.0, atol=1e-12 * pb.y1)


def test_cell_index_at_faces():
    pb = P.couette_1d(ncell=10, precision=64)
    for j in range(10):
        y = pb.y0 + j * pb.dy
        if (y - pb.y0) * pb.inv_dy >= j:
            d, r = O.advect(pb, _one([0.0, 0.0, 0.0], y), j, 0, 0)
            assert d == j


def _sort_reference(pb, st):
    """canonical order by brute force: advect every particle, then Python's
    sorted on (new cell, source displacement (row-major, minimal image), slot)"""
    per_y = pb.faces[2].kind == P.BC_PERIODIC
    per_x = pb.faces[0].kind == P.BC_PERIODIC

    def mi(d, n, per):
        if not per:
            return d
        d %= n
        return d - n if d > n - n // 2 - 1 else d

    ent = []
    off = st.offsets
    for c in range(pb.ncell):
        for s in range(st.counts[c]):
            d, r = O.advect(pb, st.parts[off[c] + s], c, s, st.step)
            sx, sy, dx_, dy_ = c % pb.nx, c // pb.nx, d % pb.nx, d // pb.nx
            ent.append(((d, mi(sy - dy_, pb.ny, per_y), mi(sx - dx_, pb.nx, per_x), s), r, d,
                        off[c] + s))
    ent.sort(key=lambda e: e[0])
    counts = np.bincount([e[2] for e in ent], minlength=pb.ncell)
    pos = np.array([[e[1][0], e[1][1]] for e in ent])
    perm = np.array([e[3] for e in ent], np.int64)
    return counts, pos, perm


@pytest.mark.parametrize("which", ["couette", "box", "cavity", "sod"])
def test_stable_sort_matches_brute_force(which):
    # With P_ne = 0 no particles are added, all weights stay 1 so no particle
    # is deleted, and relaxation never moves a particle: the positions after
    # one step are exactly the advected positions in canonical order.
    if which == "couette":
        pb = P.couette_1d(ncell=12, ppc=30, precision=32)
    elif which == "box":
        pb = P.homogeneous_box(ncell=7, ppc=40, nu_dt=1.0, precision=32)
        pb = pb.replace(dt=pb.dt * 40)  # cross several cells and the periodic face
    elif which == "sod":
        pb = P.sod_1d(ncell=16, mean_ppc=30, precision=64)
    else:
        pb = P.cavity_2d(Kn=0.05, n=6, ppc=30, precision=32)
        pb = pb.replace(dt=pb.dt * 6)
    pb = pb.replace(pne_mode=P.PNE_FIXED, pne_fixed=0.0)
    o = O.Oracle(pb)
    st = o.get_state()
    counts, pos, perm = _sort_reference(pb, st)
    assert o.get_sort() is None
    o.step(1)
    st1 = o.get_state()
    assert np.array_equal(st1.counts, counts)
    # the recorded sort: counts after it and each particle's place before it
    scnt, sperm = o.get_sort()
    assert np.array_equal(scnt, counts)
    assert np.array_equal(sperm, perm)
    if pb.dim == 2:
        assert np.array_equal(st1.parts[:, 0], pos[:, 0])
    assert np.array_equal(st1.parts[:, 1], pos[:, 1])
