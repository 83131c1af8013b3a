"""CPU: the oracle's marg_cons diagnostic, the smallest relative gap between
a value the conservation correction tests and its bound (W_r against 1/2
and 2, the mean shift against 3 rms spreads, s^2 against 1/9 and 9, the
whole-cell conditions).  A value within rounding of a bound may take either
branch, so a comparison that meets one treats the cell as a tie.  Test
diagnostics only: the step does not read them."""
import numpy as np

from oracle import oracle as O
from paper_1808_03801_amd import problems as P
from tests.test_gpu_parity_sweep import _oracle_state, draw_case


def test_the_oracle_reports_a_mass_correction_at_its_bound():
    """a random-sweep draw (an FP64 slit) whose cell 116 sums to W_r two ulps
    above 2 in the oracle: the mass correction fails there and the whole-cell
    correction takes over (flag 16), where sums in another order give 2.0
    and the ordinary correction; the gap it records is at rounding level"""
    label, pb, first, warm = draw_case(6083)
    o = O.Oracle(pb)
    o.set_state(_oracle_state(pb, warm))
    o.step(1)
    dg = o.diag()[116]
    assert abs(dg[O.DIAG["Wr"]] - 2.0) < 1e-14, label
    assert dg[O.DIAG["flags"]] == 16.0
    assert dg[O.DIAG["marg_cons"]] < 1e-14


def test_gaps_are_recorded_where_the_correction_ran():
    """every cell that reassigned particles records a finite gap in [0, 2]
    (W_r is always tested against 1/2 and 2); cells without reassigned
    particles keep none"""
    pb = P.couette_1d(Kn=0.1, ncell=40, ppc=80, precision=64, seed=5)
    o = O.Oracle(pb)
    o.step(3)
    dg = o.diag()
    m = dg[:, O.DIAG["marg_cons"]]
    ran = dg[:, O.DIAG["n_usp"]] > 0
    assert ran.any()
    assert np.all(np.isfinite(m[ran])) and np.all((m[ran] >= 0) & (m[ran] <= 2))
    assert np.all(np.isinf(m[~ran]))
