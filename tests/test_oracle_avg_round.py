"""Pins of the Eq. 34 time average and of the Eq. 28 rounding.

Eq. 34 (Section 3.2.3): Q^{n+1} = (1 - 1/n_a) Q^n + Q_sample / n_a, here on the
raw per-cell sums.  A single periodic cell of hard-sphere gas under a uniform
body acceleration a along x, with P_ne = 0 (no added particles), keeps its
mass exactly (every selected particle has weight 1, so Eq. 28 reassigns all
of them) and, with the conservation correction restoring the momentum of
f-tilde^*, gains exactly M a dt of x momentum per step: the sample of step
k is S_k = S_0 + k d, d = M a dt.  The recursion then has closed forms,
written here as solutions (not as the recursion):
  * start from the first sample with a running mean while k <= n_a:
    A_k = S_0 + d (k + 1) / 2;  beyond, with r = 1 - 1/n_a and B = A - S:
    B_k = B* + r^(k - n_a) (B_{n_a} - B*),  B* = -(n_a - 1) d;
  * start from the exact initial moments (here 0 for the momentum) with the
    fixed window from the first step: B_k = B* + r^k (B_0 - B*), B_0 = -S_0.
A window weight off by one sample (1 / (n_a + 1)) moves B* by d, a start
one step late shifts the running mean by d / 2: both far outside 1e-9.

Eq. 28 (Section 3.2.2): N_usp = int(sum of the selected weights), int the
nearest integer (the paper's own definition for Eq. 9).  With added
particles of non-integer weight the selected sum S is not an integer; the
mass change N_usp - S of a cell is then in [-1/2, 1/2] and its mean over
many cells is 0 (floor rounding gives values in (-1, 0] and a mean of -1/2;
ceiling, [0, 1) and +1/2).
"""
import math

import numpy as np

from oracle import oracle as O
from paper_1808_03801_amd import problems as P

S1X = 13 + 1      # raw sum of w c_x in the state record
A1X = 2 * 13 + 1  # its Eq. 34 average


def _accelerated_cell(avg_init, n_avg, accel=2.0e9, ppc=400, seed=3):
    pb = P.homogeneous_box(ncell=1, ppc=ppc, nu_dt=0.5, precision=64, pne=0.0, seed=seed)
    return pb.replace(accel=(accel, 0.0, 0.0), n_avg=n_avg, avg_init=avg_init,
                      jmom_mode=P.JMOM_INST)


def _run(pb, steps):
    o = O.Oracle(pb)
    s0 = o.get_state()
    M = s0.cells[0, 13]
    S0 = s0.cells[0, S1X]
    raw, avg = [], []
    for _ in range(steps):
        assert o.step(1) == 0
        st = o.get_state()
        raw.append(st.cells[0, S1X])
        avg.append(st.cells[0, A1X])
        assert st.cells[0, 13] == M  # mass kept exactly
    return M, S0, np.array(raw), np.array(avg)


def test_body_force_adds_exactly_M_a_dt_per_step():
    pb = _accelerated_cell(0, 20)
    M, S0, raw, _ = _run(pb, 30)
    d = M * pb.accel[0] * pb.dt
    k = np.arange(1, 31)
    assert np.allclose(raw, S0 + k * d, rtol=0, atol=1e-9 * 30 * abs(d))


def test_eq34_running_mean_then_exponential_window():
    n = 20
    pb = _accelerated_cell(0, n)
    M, S0, raw, avg = _run(pb, 70)
    d = M * pb.accel[0] * pb.dt
    k = np.arange(1, 71)
    S = S0 + k * d
    expect = np.empty(70)
    run = k <= n
    expect[run] = S0 + d * (k[run] + 1) / 2.0
    r = 1.0 - 1.0 / n
    Bstar = -(n - 1) * d
    Bn = -d * (n - 1) / 2.0
    B = Bstar + r ** (k[~run] - n) * (Bn - Bstar)
    expect[~run] = S[~run] + B
    assert np.allclose(avg, expect, rtol=0, atol=1e-9 * n * abs(d))
    # the lag behind the sample approaches -(n_a - 1) d
    assert abs((avg[-1] - raw[-1]) / Bstar - 1.0) < 0.1


def test_eq34_fixed_window_from_the_initial_moments():
    n = 15
    pb = _accelerated_cell(1, n)
    M, S0, raw, avg = _run(pb, 50)
    d = M * pb.accel[0] * pb.dt
    k = np.arange(1, 51)
    r = 1.0 - 1.0 / n
    Bstar = -(n - 1) * d
    B0 = 0.0 - S0  # initial Maxwellian at rest: its momentum sum is exactly 0
    expect = S0 + k * d + Bstar + r ** k * (B0 - Bstar)
    assert np.allclose(avg, expect, rtol=0, atol=1e-9 * (n * abs(d) + abs(S0)))


def test_eq28_nearest_integer_leaves_no_mass_bias():
    # weighted step-4 particles make the selected sum non-integer; without
    # the conservation correction N_usp - S is the cell's mass change
    pb = P.thermal_couette_1d(Kn=1e-2, ncell=200, ppc=100, precision=64, seed=11)
    pb = pb.replace(conserve_mode=P.CONSERVE_NONE, pne_mode=P.PNE_FIXED, pne_fixed=1.0,
                    jmom_mode=P.JMOM_AVG, spawn_projection=0)
    o = O.Oracle(pb)
    diffs = []
    for _ in range(25):
        assert o.step(1) == 0
        dg = o.diag()
        S = dg[:, O.DIAG["s_sel"]]
        nusp = dg[:, O.DIAG["n_usp"]]
        nsel = dg[:, O.DIAG["n_sel"]]
        free = (S > 0.5) & (S < nsel - 0.5)  # the clamp to [0, N_s] does not act
        diffs.append((nusp - S)[free])
    dd = np.concatenate(diffs)
    assert dd.size > 3000
    frac = dd - np.floor(dd)
    assert np.ptp(frac) > 0.9  # S really takes non-integer values
    assert np.all(np.abs(dd) <= 0.5 + 1e-9)
    se = dd.std() / math.sqrt(dd.size)
    assert abs(dd.mean()) < 3.0 * se + 1e-3, (dd.mean(), se)
