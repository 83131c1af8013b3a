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


def compare_step(pb, st_o, st_g, dg_o, dg_g, f_o, f_g, report=None):
    """Returns a dict of mismatch counts; raises AssertionError with details
    when the bar is not met."""
    nc = pb.ncell
    ties = tie_cells(dg_o)
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
    # particles of matching cells, element by element
    oo, og = st_o.offsets, st_g.offsets
    th = pb.gas.R * 273.0
    sq = math.sqrt(th)
    if pb.precision == 32:
        tol_x = 4e-7 * max(abs(pb.y1), abs(pb.x1 if pb.dim == 2 else 0))
        tol_c = 2e-5 * sq
        tol_w = 2e-5
    else:
        tol_x = 1e-12 * abs(pb.y1)
        tol_c = 1e-9 * sq
        tol_w = 1e-9
    worst = dict(x=0.0, c=0.0, w=0.0)
    for c in np.nonzero(ok)[0]:
        a = st_o.parts[oo[c]:oo[c + 1]]
        b = st_g.parts[og[c]:og[c + 1]]
        dx = np.abs(a[:, :2] - b[:, :2]).max(initial=0.0)
        dc = np.abs(a[:, 2:5] - b[:, 2:5]).max(initial=0.0)
        dw = (np.abs(a[:, 5] - b[:, 5]) / np.maximum(1.0, np.abs(a[:, 5]))).max(initial=0.0)
        worst["x"] = max(worst["x"], dx)
        worst["c"] = max(worst["c"], dc)
        worst["w"] = max(worst["w"], dw)
        assert dx <= tol_x, f"cell {c}: position differs by {dx}"
        assert dc <= tol_c, f"cell {c}: velocity differs by {dc}"
        assert dw <= tol_w, f"cell {c}: weight differs by {dw}"
    # moments per cell
    rho, T, p = f_o[:, 1], f_o[:, 5], f_o[:, 6]
    valid = ok & (p > 0)
    sth = np.sqrt(np.where(valid, p / np.where(rho > 0, rho, 1.0), 1.0))
    rel = {}
    rel["rho"] = np.abs(f_g[:, 1] - rho) / np.abs(rho)
    rel["u"] = np.abs(f_g[:, 2:5] - f_o[:, 2:5]).max(1) / sth
    rel["T"] = np.abs(f_g[:, 5] - T) / np.abs(T)
    rel["sigma"] = np.abs(f_g[:, 7:13] - f_o[:, 7:13]).max(1) / p
    rel["q"] = np.abs(f_g[:, 13:16] - f_o[:, 13:16]).max(1) / (p * sth)
    out = {}
    for k, v in rel.items():
        m = float(np.max(v[valid], initial=0.0))
        out[k] = m
        assert m <= 1e-5, f"moment {k}: max relative error {m}"
    out.update(mismatched_cells=int(bad_int.sum()), tie_cells=int(ties.sum()), **worst)
    if report is not None:
        report.update(out)
    return out
