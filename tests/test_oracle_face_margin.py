"""CPU: the oracle's marg_face diagnostic (the smallest distance of a
landing point of a step's flights to a face two cells share, kept in both
cells), which lets a comparison over several steps recognise a particle
that the rounding of its flight may put on either side of a face.  Checked
against a replay of the step's flights through the oracle's single-particle
advection: the recorded margin is never above the replayed one (the step's
added particles fly too and can only lower it) and equals it in most
cells.  Test diagnostics only: the step does not read them."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1808_03801_amd import problems as P


def _shared_face(pb, d, x, y):
    """(distance, other cell) of the nearest face of cell d that another
    cell shares, or (inf, -1)"""
    nx, ny = pb.nx, pb.ny
    ix, iy = d % nx, d // nx
    best, other = np.inf, -1
    axes = [(0, x, pb.x0, pb.dx, ix, nx), (1, y, pb.y0, pb.dy, iy, ny)]
    for a, pos, org, h, i, n in axes[(0 if pb.dim == 2 else 1):]:
        periodic = pb.faces[2 * a].kind == P.BC_PERIODIC
        for sd in (0, 1):
            j = i + (1 if sd else -1)
            if j < 0 or j >= n:
                if not periodic or n == 1:
                    continue
                j %= n
            dist = abs(pos - (org + (i + sd) * h))
            if dist < best:
                best, other = dist, (iy * nx + j if a == 0 else j * nx + ix)
    return best, other


@pytest.mark.parametrize("make", [
    lambda: P.cavity_2d(Kn=0.01, n=8, ppc=40, precision=64, seed=3),
    lambda: P.homogeneous_box(ncell=6, ppc=60, precision=64, seed=4),
], ids=["cavity_walls", "periodic_box"])
def test_face_margin_matches_a_replay_of_the_flights(make):
    pb = make()
    o = O.Oracle(pb)
    o.step(2)
    st = o.get_state()
    o.step(1)
    assert o.error == 0
    got = o.diag()[:, O.DIAG["marg_face"]]
    rep = np.full(pb.ncell, np.inf)
    off = st.offsets
    for c in range(pb.ncell):
        for s in range(st.counts[c]):
            d, r = O.advect(pb, st.parts[off[c] + s], c, s, st.step)
            if d < 0:
                continue
            dist, other = _shared_face(pb, d, r[0], r[1])
            if other >= 0:
                rep[d] = min(rep[d], dist)
                rep[other] = min(rep[other], dist)
    assert np.all(got <= rep), np.nonzero(got > rep)[0]
    assert np.mean(got == rep) >= 0.5, (got, rep)
    # a margin is a distance inside a cell: never above half its size
    assert np.all(got <= 0.5 * max(pb.dy, pb.dx if pb.dim == 2 else 0.0) + 1e-300)
