"""Comparison helpers for GPU-vs-oracle parity tests.

Protocol (single step, re-synchronised): the oracle produces a state; the
same state is loaded into a fresh oracle and into the GPU library; both take
one step; then
  * per-cell counts and every integer decision of the step (added, selected,
    reassigned, deleted counts) must be identical, except in cells where the
    oracle reports a decision within `TIE` of its threshold;
  * particles of matching cells are compared element by element (canonical
    order, so this also checks the sort permutation);
  * moments are compared per cell within 1e-5 relative to their natural
    scale (rho for rho, sqrt(theta) for u, T for T, p for sigma, p sqrt(theta)
    for q).
"""
import math

import numpy as np

from oracle import oracle as O

INT_DIAG = ["n_in", "n4", "n_sel", "n_usp", "n_del", "n7", "n_out", "n2", "n_inj", "n_gone"]
TIE = 1e-9


def tie_cells(dg_oracle):
    d = dg_oracle
    m = np.minimum.reduce([d[:, O.DIAG["marg_sel"]], d[:, O.DIAG["marg_round"]],
                           d[:, O.DIAG["marg_cnt"]], d[:, O.DIAG["marg_cnt2"]]])
    return m < TIE


def value_tie_cells(dg_oracle, precision):
    """cells whose conservation correction tested a value (W_r, the mean
    shift, s^2, the whole-cell conditions) within a relative gap of its
    bound that the rounding of its sums can cross (FP64 sums of particles
    of the state precision): either branch is correct, the counts are the
    same and the values are not, so such a cell is compared on its integer
    decisions only"""
    return dg_oracle[:, O.DIAG["marg_cons"]] < (1e-5 if precision == 32 else 1e-9)


def degenerate_cells(dg_oracle, f_oracle):
    """cells the step leaves without valid moments: the oracle skipped their
    relaxation (f-tilde^* of non-positive mass or temperature) or their
    result has non-positive density or temperature.  Weights of either sign
    cancel there, so a rounding of the state precision is amplified by the
    ratio of sum |W| to |sum W| in every value the cell produces; their counts
    and integer decisions are compared, their values are not."""
    F_SKIP = 1
    flags = dg_oracle[:, O.DIAG["flags"]].astype(np.int64)
    return ((flags & F_SKIP) != 0) | ~(f_oracle[:, 1] > 0.0) | ~(f_oracle[:, 5] > 0.0)


def _abs_weight_scales(pb, st_o, f_o):
    """per cell: the density and temperature of the cell's particles with
    every weight taken positive (rho f_o scaled by sum |W| / |sum W|; the
    thermal energy about the cell's velocity over 3 R sum |W|)"""
    nc = pb.ncell
    counts = st_o.counts
    cell = np.repeat(np.arange(nc), counts)
    w = np.abs(st_o.parts[:, 5])
    u = f_o[cell, 2:5]
    C2 = ((st_o.parts[:, 2:5] - u) ** 2).sum(1)
    Wabs = np.bincount(cell, weights=w, minlength=nc)
    Wsum = np.bincount(cell, weights=st_o.parts[:, 5], minlength=nc)
    Eabs = np.bincount(cell, weights=w * C2, minlength=nc)
    with np.errstate(invalid="ignore", divide="ignore"):
        rho_abs = np.where(np.abs(Wsum) > 0, np.abs(f_o[:, 1]) * Wabs / np.abs(Wsum), 0.0)
        T_abs = np.where(Wabs > 0, Eabs / (3.0 * pb.gas.R * Wabs), 0.0)
    return rho_abs, T_abs


def dilate(pb, mask, k):
    """cells within k cells (each axis) of a cell of mask"""
    m = mask.reshape(pb.ny, pb.nx)
    out = m.copy()
    per_y = pb.faces[2].kind == 2
    per_x = pb.faces[0].kind == 2
    for dy in range(-k, k + 1):
        for dx in range(-k, k + 1):
            if pb.dim == 1 and dx != 0:
                continue
            sh = np.roll(m, (dy, dx), axis=(0, 1))
            if not per_y:
                if dy > 0:
                    sh[:dy, :] = False
                elif dy < 0:
                    sh[dy:, :] = False
            if not per_x:
                if dx > 0:
                    sh[:, :dx] = False
                elif dx < 0:
                    sh[:, dx:] = False
            out |= sh
    return out.reshape(-1)


def _cell_scales(cells_o):
    """per-cell scales of the four 13-moment blocks of a state record: mass
    M, thermal speed v, and the bulk speed U of the cell"""
    mom = cells_o[:, :13]
    M = np.abs(cells_o[:, 13])
    trK = mom[:, 4] + mom[:, 5] + mom[:, 6]
    ok = (M > 0) & (trK > 0)
    th = np.where(ok, trK / (3.0 * np.where(M > 0, M, 1.0)), 1.0)
    v = np.sqrt(th)
    U = np.sqrt((mom[:, 1:4] ** 2).sum(1))
    return ok, M, v, U


def compare_cells(pb, st_o, st_g, cells_ok, tol=1e-5):
    """the per-cell records of the two states (centred moments, raw sums, the
    Eq. 34 averages of f^n and of f-tilde^*, P_ne^n, P_ne^{n-1}), relative to
    the natural scale of each moment; P_ne absolutely.  Returns the largest
    error per block."""
    co, cg = st_o.cells, st_g.cells
    ok, M, v, U = _cell_scales(co)
    use = cells_ok & ok
    s_raw = np.empty((co.shape[0], 13))
    s_raw[:, 0] = M
    s_raw[:, 1:4] = (M * (U + v))[:, None]
    s_raw[:, 4:10] = (M * (U * U + v * v))[:, None]
    s_raw[:, 10:13] = (M * (U * U + v * v) ** 1.5)[:, None]
    s_cen = np.empty_like(s_raw)
    s_cen[:, 0] = M
    s_cen[:, 1:4] = v[:, None]
    s_cen[:, 4:10] = (M * v * v)[:, None]
    s_cen[:, 10:13] = (M * v ** 3)[:, None]
    out = {}
    for name, b, sc in (("mom", 0, s_cen), ("raw", 1, s_raw), ("avg", 2, s_raw),
                        ("avgs", 3, s_raw)):
        # a moment far above its natural scale (a degenerate cell: weights of
        # either sign, a trace of K far below its diagonal) is compared
        # relative to its own size
        sc = np.maximum(sc, np.abs(co[:, 13 * b:13 * b + 13]))
        # empty cells have no scale (0 / 0); they are not in `use`, and a NaN
        # in a used cell fails the bar (the max is NaN)
        with np.errstate(invalid="ignore", divide="ignore"):
            d = np.abs(co[:, 13 * b:13 * b + 13] - cg[:, 13 * b:13 * b + 13]) / sc
        m = float(np.max(d[use], initial=0.0))
        out["cells_" + name] = m
        assert m <= tol, f"cell record {name}: max relative error {m}"
    for name, i in (("pne", 52), ("pne_prev", 53)):
        d = np.abs(co[:, i] - cg[:, i])
        m = float(np.max(d[cells_ok], initial=0.0))
        out[name] = m
        assert m <= tol, f"{name}: max difference {m}"
    return out


def compare_step(pb, st_o, st_g, dg_o, dg_g, f_o, f_g, report=None, excuse=None,
                 excuse_values=None, steps=1):
    """Returns a dict of mismatch counts; raises AssertionError with details
    when the bar is not met.  excuse: cells whose integer decisions may
    differ for a reason outside this step (a tie of an earlier step in
    reach of them); excuse_values: cells whose values may differ for such a
    reason (a degenerate cell of an earlier step in reach of them).  Cells
    with particles whose values the step leaves degenerate
    (degenerate_cells) are compared on their integer decisions only.
    steps: time steps since the common state; the value bars are that many
    times the one-step bars (the first step's rounding reaches the next
    step's cell scalars through the moments, and from there every resampled
    and added particle: to first order the differences add up)."""
    nc = pb.ncell
    th = pb.gas.R * 273.0
    sq = math.sqrt(th)
    # positions: a few roundings of the larger of the domain size and the
    # longest flight of the step (a flight of several domain lengths between
    # walls carries the rounding of the distance flown); over several steps
    # also the velocity difference an earlier relaxation left (within the
    # velocity bar, on the larger of sqrt(theta) and the particle's speed),
    # flown for dt in each later step
    vmax = float(np.abs(st_o.parts[:, 2:5]).max(initial=0.0)) * math.sqrt(3.0)
    L = max(abs(pb.y1), abs(pb.x1 if pb.dim == 2 else 0), vmax * pb.dt)
    flown = (steps - 1) * max(sq, vmax) * pb.dt
    if pb.precision == 32:
        tol_x = 4e-7 * L + 2e-5 * flown
        tol_c = 2e-5 * sq * steps
        tol_w = 2e-5 * steps
    else:
        # a projected batch of a few particles solves a Gram system whose
        # condition number (up to 1e10 by its pivot test) multiplies the
        # rounding of its inputs; the cell its particles fly to takes their
        # weights into the mass, momentum and energy of its conservation
        # correction, which passes the difference on to the weight and the
        # velocity of every particle it reassigns
        rel = 1e-6 if pb.spawn_projection == 1 else 1e-9
        tol_x = 1e-12 * L + rel * flown
        tol_c = rel * sq * steps
        tol_w = rel * steps
    ties = tie_cells(dg_o)
    if excuse is not None:
        ties = ties | excuse
    if steps > 1:
        # a flight of a later step starts from velocities that differ within
        # their bar, so one that ends within the position bar of a face two
        # cells share may end on either side of it (the oracle keeps that
        # distance in both cells)
        ties = ties | (dg_o[:, O.DIAG["marg_face"]] < tol_x)
    # a decision that flips in one cell moves particles of its neighbours only
    # through the next step, so the cells themselves are the unit of comparison
    bad_int = np.zeros(nc, bool)
    for k in INT_DIAG:
        bad_int |= dg_o[:, O.DIAG[k]] != dg_g[:, O.DIAG[k]]
    bad_int |= st_o.counts != st_g.counts
    unexplained = bad_int & ~ties
    assert not unexplained.any(), (
        f"integer mismatch in cells {np.nonzero(unexplained)[0][:10]}: "
        + "; ".join(f"{k} o={dg_o[c, O.DIAG[k]]} g={dg_g[c, O.DIAG[k]]}"
                    for c in np.nonzero(unexplained)[0][:2] for k in INT_DIAG
                    if dg_o[c, O.DIAG[k]] != dg_g[c, O.DIAG[k]]))
    ok = ~bad_int
    deg = degenerate_cells(dg_o, f_o) | value_tie_cells(dg_o, pb.precision)
    deg &= st_o.counts > 0
    if excuse_values is not None:
        deg = deg | excuse_values
    # particles of matching cells, element by element
    oo, og = st_o.offsets, st_g.offsets
    worst = dict(x=0.0, c=0.0, w=0.0)
    for c in np.nonzero(ok & ~deg)[0]:
        a = st_o.parts[oo[c]:oo[c + 1]]
        b = st_g.parts[og[c]:og[c + 1]]
        dx = np.abs(a[:, :2] - b[:, :2]).max(initial=0.0)
        # velocities on the larger of the reference thermal speed and the
        # particle's own speed (a tail particle of 14 sqrt(theta) carries the
        # rounding of its own magnitude)
        dc = (np.abs(a[:, 2:5] - b[:, 2:5]) /
              np.maximum(1.0, np.abs(a[:, 2:5]) / sq)).max(initial=0.0)
        dw = (np.abs(a[:, 5] - b[:, 5]) / np.maximum(1.0, np.abs(a[:, 5]))).max(initial=0.0)
        worst["x"] = max(worst["x"], dx)
        worst["c"] = max(worst["c"], dc)
        worst["w"] = max(worst["w"], dw)
        assert dx <= tol_x, f"cell {c}: position differs by {dx}"
        assert dc <= tol_c, f"cell {c}: velocity differs by {dc}"
        assert dw <= tol_w, f"cell {c}: weight differs by {dw}"
    # moments per cell
    rho, T, p = f_o[:, 1], f_o[:, 5], f_o[:, 6]
    valid = ok & ~deg & (p > 0)
    sth = np.sqrt(np.where(valid, p / np.where(rho > 0, rho, 1.0), 1.0))
    # density and temperature relative to their values, or to the values the
    # cell's particles would give with all weights taken positive where
    # weights of either sign cancel (a cell at 0.17 K of particles at
    # hundreds of m/s): the rounding scales with sum |W|, not |sum W|
    rho_abs, T_abs = _abs_weight_scales(pb, st_o, f_o)
    rel = {}
    rel["rho"] = np.abs(f_g[:, 1] - rho) / np.maximum(np.abs(rho), rho_abs)
    rel["u"] = np.abs(f_g[:, 2:5] - f_o[:, 2:5]).max(1) / sth
    rel["T"] = np.abs(f_g[:, 5] - T) / np.maximum(np.abs(T), T_abs)
    # stress and heat flux on their natural scales p and p sqrt(theta), or
    # on their own size in a degenerate cell where that is larger (weights
    # of either sign: a heat flux of 500 p sqrt(theta) has been drawn)
    # (an empty cell has both scales 0; only valid cells, where they are
    # positive, are read below, and a NaN there fails the bar)
    s_sig = np.maximum(p, np.abs(f_o[:, 7:13]).max(1))
    s_q = np.maximum(p * sth, np.abs(f_o[:, 13:16]).max(1))
    with np.errstate(invalid="ignore", divide="ignore"):
        rel["sigma"] = np.abs(f_g[:, 7:13] - f_o[:, 7:13]).max(1) / s_sig
        rel["q"] = np.abs(f_g[:, 13:16] - f_o[:, 13:16]).max(1) / s_q
    # over several steps a cell's moments also carry the weight differences
    # of the particles that arrived from the earlier steps (within the
    # one-step weight bar): the relaxation conserves the mass, momentum and
    # energy those weights sum to
    tol_m = 1e-5 * steps + (steps - 1) * tol_w / steps
    out = {}
    for k, v in rel.items():
        m = float(np.max(v[valid], initial=0.0))
        out[k] = m
        assert m <= tol_m, f"moment {k}: max relative error {m}"
    # P_ne and the averages: a cell's P_ne reads its neighbours' moments
    kk = 1
    near_bad = dilate(pb, bad_int | deg, kk)
    pne_rel = np.abs(f_g[:, 16] - f_o[:, 16])
    out["pne_field"] = float(np.max(pne_rel[~near_bad], initial=0.0))
    assert out["pne_field"] <= 1e-5, f"P_ne: max difference {out['pne_field']}"
    out.update(compare_cells(pb, st_o, st_g, ~near_bad, tol=tol_m))
    out.update(mismatched_cells=int(bad_int.sum()), tie_cells=int(ties.sum()),
               degenerate_cells=int(deg.sum()), **worst)
    if report is not None:
        report.update(out)
    return out
