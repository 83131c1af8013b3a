"""Exact solution of the Riemann problem of the Euler equations for an ideal
gas (the textbook construction: a pressure p* between the two initial states
from the shock / rarefaction relations, solved by Newton iteration, then the
self-similar wave fan sampled at x/t).  Test infrastructure: the continuum
limit that the Sod tube of Section 4.3 approaches at small Kn."""
import math

import numpy as np


def _f(p, rho, pk, a, g):
    """velocity jump across the wave that takes state (rho, pk) to pressure p,
    and its derivative in p"""
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        s = math.sqrt(A / (p + B))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (p + B))
    # rarefaction
    r = (p / pk) ** ((g - 1.0) / (2.0 * g))
    return 2.0 * a / (g - 1.0) * (r - 1.0), (p / pk) ** (-(g + 1.0) / (2.0 * g)) / (rho * a)


def star_state(left, right, g):
    """(p*, u*) of the Riemann problem (rho, u, p) left | right"""
    rl, ul, pl = left
    rr, ur, pr = right
    al, ar = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    p = max(1e-12 * (pl + pr), 0.5 * (pl + pr))
    for _ in range(100):
        fl, dl = _f(p, rl, pl, al, g)
        fr, dr = _f(p, rr, pr, ar, g)
        dp = (fl + fr + ur - ul) / (dl + dr)
        p_new = max(p - dp, 1e-12 * (pl + pr))
        if abs(p_new - p) < 1e-14 * (p_new + p):
            p = p_new
            break
        p = p_new
    fl, _ = _f(p, rl, pl, al, g)
    fr, _ = _f(p, rr, pr, ar, g)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def sample(xi, left, right, g):
    """(rho, u, p) at x / t = xi for every entry of the array xi"""
    rl, ul, pl = left
    rr, ur, pr = right
    al, ar = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    ps, us = star_state(left, right, g)
    out = np.zeros((len(xi), 3))
    for i, s in enumerate(np.asarray(xi, float)):
        if s <= us:  # left of the contact
            if ps > pl:  # left shock
                sl = ul - al * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if s <= sl:
                    out[i] = (rl, ul, pl)
                else:
                    r = rl * (ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1)
                    out[i] = (r, us, ps)
            else:  # left rarefaction
                head = ul - al
                a_s = al * (ps / pl) ** ((g - 1) / (2 * g))
                tail = us - a_s
                if s <= head:
                    out[i] = (rl, ul, pl)
                elif s >= tail:
                    out[i] = (rl * (ps / pl) ** (1 / g), us, ps)
                else:
                    c = 2 / (g + 1) + (g - 1) / ((g + 1) * al) * (ul - s)
                    out[i] = (rl * c ** (2 / (g - 1)), 2 / (g + 1) * (al + (g - 1) / 2 * ul + s),
                              pl * c ** (2 * g / (g - 1)))
        else:  # right of the contact
            if ps > pr:  # right shock
                sr = ur + ar * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                if s >= sr:
                    out[i] = (rr, ur, pr)
                else:
                    r = rr * (ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1)
                    out[i] = (r, us, ps)
            else:  # right rarefaction
                head = ur + ar
                a_s = ar * (ps / pr) ** ((g - 1) / (2 * g))
                tail = us + a_s
                if s >= head:
                    out[i] = (rr, ur, pr)
                elif s <= tail:
                    out[i] = (rr * (ps / pr) ** (1 / g), us, ps)
                else:
                    c = 2 / (g + 1) - (g - 1) / ((g + 1) * ar) * (ur - s)
                    out[i] = (rr * c ** (2 / (g - 1)), 2 / (g + 1) * (-ar + (g - 1) / 2 * ur + s),
                              pr * c ** (2 * g / (g - 1)))
    return out
