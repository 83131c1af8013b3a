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


def check_profiles(z, names, frac_within=0.99, hard=5.0):
    """every field: at least frac_within of the cells inside 3 sigma and
    none beyond `hard` sigma.  Also reported: the cell-averaged z times
    sqrt(ncell), a bias common to the whole profile (not asserted: the cells
    of a profile are correlated)."""
    ncell = z.shape[0]
    report = {}
    for k, name in enumerate(names):
        zk = z[:, k]
        inside = float(np.mean(np.abs(zk) <= 3.0))
        worst = float(np.max(np.abs(zk)))
        bias = float(np.mean(zk) * np.sqrt(ncell))
        report[name] = dict(inside_3sigma=inside, max_abs_z=worst, mean_z_scaled=bias)
        assert inside >= frac_within, (name, report[name])
        assert worst <= hard, (name, report[name])
    return report
