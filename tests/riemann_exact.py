"""Exact solution of the one-dimensional Riemann problem for an ideal gas
(textbook two-shock/two-rarefaction star-state iteration, Toro, "Riemann
Solvers and Numerical Methods for Fluid Dynamics", ch. 4)."""
import math

import numpy as np


def _fk(p, rk, pk, ck, g):
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rk)
        Bk = (g - 1.0) / (g + 1.0) * pk
        f = (p - pk) * math.sqrt(A / (p + Bk))
        df = math.sqrt(A / (Bk + p)) * (1.0 - 0.5 * (p - pk) / (Bk + p))
    else:  # rarefaction
        f = 2.0 * ck / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rk * ck) * (p / pk) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(rl, ul, pl, rr, ur, pr, g):
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    p = max(1e-12, 0.5 * (pl + pr))
    for _ in range(200):
        fl, dfl = _fk(p, rl, pl, cl, g)
        fr, dfr = _fk(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(1e-14, p - dp)
        if abs(pn - p) / (0.5 * (pn + p)) < 1e-15:
            p = pn
            break
        p = pn
    fl, _ = _fk(p, rl, pl, cl, g)
    fr, _ = _fk(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(xi, rl, ul, pl, rr, ur, pr, g):
    """density, velocity, pressure at similarity coordinate xi = x / t."""
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    ps, us = star_state(rl, ul, pl, rr, ur, pr, g)
    gm = (g - 1.0) / (g + 1.0)
    out = np.zeros((3, len(xi)))
    for k, s in enumerate(xi):
        if s <= us:  # left of contact
            if ps > pl:
                sl = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if s <= sl:
                    r, u, p = rl, ul, pl
                else:
                    r = rl * (ps / pl + gm) / (gm * ps / pl + 1.0)
                    u, p = us, ps
            else:
                shl = ul - cl
                csl = cl * (ps / pl) ** ((g - 1) / (2 * g))
                stl = us - csl
                if s <= shl:
                    r, u, p = rl, ul, pl
                elif s >= stl:
                    r = rl * (ps / pl) ** (1.0 / g)
                    u, p = us, ps
                else:
                    u = 2.0 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    c = 2.0 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    r = rl * (c / cl) ** (2.0 / (g - 1))
                    p = pl * (c / cl) ** (2.0 * g / (g - 1))
        else:
            if ps > pr:
                sr = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                if s >= sr:
                    r, u, p = rr, ur, pr
                else:
                    r = rr * (ps / pr + gm) / (gm * ps / pr + 1.0)
                    u, p = us, ps
            else:
                shr = ur + cr
                csr = cr * (ps / pr) ** ((g - 1) / (2 * g))
                str_ = us + csr
                if s >= shr:
                    r, u, p = rr, ur, pr
                elif s <= str_:
                    r = rr * (ps / pr) ** (1.0 / g)
                    u, p = us, ps
                else:
                    u = 2.0 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    c = 2.0 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    r = rr * (c / cr) ** (2.0 / (g - 1))
                    p = pr * (c / cr) ** (2.0 * g / (g - 1))
        out[:, k] = (r, u, p)
    return out
