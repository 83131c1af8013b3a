"""Time-averaged profile comparison within statistical error.

Two independent runs of a steady problem (GPU against oracle: their FP32 and
FP64 trajectories part after a few decisions flip) are compared on their
time-averaged cell fields.  The statistical error of each average comes from
batch means: the averaging window is cut into `nbatch` consecutive batches,
long against the flow's correlation time, and the standard error of the mean
is the spread of the batch means over sqrt(nbatch).  The difference of the
two averages in a cell is then measured in units of its own sigma,
z = (a - b) / sqrt(se_a^2 + se_b^2).
"""
import numpy as np


def batch_stats(samples, nbatch=20):
    """samples [nsteps, ncell, nf] -> (mean [ncell, nf], standard error)"""
    s = np.asarray(samples)
    n = (s.shape[0] // nbatch) * nbatch
    b = s[:n].reshape(nbatch, n // nbatch, *s.shape[1:]).mean(axis=1)
    return b.mean(axis=0), b.std(axis=0, ddof=1) / np.sqrt(nbatch)


def z_scores(a, b, nbatch=20):
    ma, sa = batch_stats(a, nbatch)
    mb, sb = batch_stats(b, nbatch)
    se = np.sqrt(sa * sa + sb * sb)
    return (ma - mb) / np.where(se > 0, se, np.inf), ma, mb, se


def check_profiles(z, names, nbatch=20, alpha=1e-3, hard=5.0):
    """every field: the number of cells beyond 3 sigma within what chance
    allows, and none beyond `hard` sigma.

    With `nbatch` batch means each standard error has nbatch - 1 degrees of
    freedom, so z is (conservatively) Student-t with nu = nbatch - 1: a cell
    lies beyond 3 sigma with p = P(|t_nu| > 3) (0.74 % at nu = 19).  The
    count over n cells may not exceed the binomial (n, p) quantile at
    1 - alpha (at most 3 of 50 cells, 7 of 256).  Reported, not asserted
    (the cells of a profile are correlated, so neither has a known spread):
    the mean of z^2 against its expectation nu / (nu - 2) for independent
    cells, with the bound that independence would give (4 standard errors,
    variance of t^2 2 nu^2 (nu - 1) / ((nu - 2)^2 (nu - 4))), and the
    cell-averaged z times sqrt(ncell), a bias common to the whole profile."""
    from scipy import stats
    nu = nbatch - 1
    p3 = 2.0 * stats.t.sf(3.0, nu)
    e2 = nu / (nu - 2.0)
    v2 = 2.0 * nu * nu * (nu - 1.0) / ((nu - 2.0) ** 2 * (nu - 4.0))
    ncell = z.shape[0]
    allowed = int(stats.binom.ppf(1.0 - alpha, ncell, p3))
    zmax2 = e2 + 4.0 * np.sqrt(v2 / ncell)
    report = {}
    for k, name in enumerate(names):
        zk = z[:, k]
        beyond = int(np.sum(np.abs(zk) > 3.0))
        worst = float(np.max(np.abs(zk)))
        mz2 = float(np.mean(zk * zk))
        bias = float(np.mean(zk) * np.sqrt(ncell))
        report[name] = dict(beyond_3sigma=beyond, allowed=allowed, mean_z2=mz2,
                            mean_z2_max=zmax2, max_abs_z=worst, mean_z_scaled=bias)
        assert beyond <= allowed, (name, report[name])
        assert worst <= hard, (name, report[name])
    return report
