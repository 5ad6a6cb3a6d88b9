"""Exact solution of the one-dimensional Euler Riemann problem (ideal gas),
written from the textbook two-rarefaction / two-shock pressure function
(Toro, "Riemann Solvers and Numerical Methods for Fluid Dynamics", ch. 4).
Independent of the MHD oracle: used to pin it in the B = 0 limit."""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


def _f(p, rho, pk, ck, g):
    if p > pk:
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        return (p - pk) * math.sqrt(A / (p + B))
    return 2.0 * ck / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)


def star_state(rl, ul, pl, rr, ur, pr, g):
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    fn = lambda p: _f(p, rl, pl, cl, g) + _f(p, rr, pr, cr, g) + ur - ul
    ps = brentq(fn, 1e-12, 100.0 * max(pl, pr), xtol=1e-15, rtol=1e-15, maxiter=500)
    us = 0.5 * (ul + ur) + 0.5 * (_f(ps, rr, pr, cr, g) - _f(ps, rl, pl, cl, g))
    return ps, us


def sample(xi, rl, ul, pl, rr, ur, pr, g):
    """(rho, u, p) at similarity coordinates xi = x/t (array)."""
    ps, us = star_state(rl, ul, pl, rr, ur, pr, g)
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    gm = (g - 1.0) / (g + 1.0)
    for n, s in enumerate(xi):
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                rs = rl * ((ps / pl + gm) / (gm * ps / pl + 1.0))
                sl = ul - cl * math.sqrt((g + 1.0) / (2 * g) * ps / pl + (g - 1.0) / (2 * g))
                st = (rl, ul, pl) if s < sl else (rs, us, ps)
            else:  # left rarefaction
                rs = rl * (ps / pl) ** (1.0 / g)
                cs = cl * (ps / pl) ** ((g - 1.0) / (2 * g))
                if s < ul - cl:
                    st = (rl, ul, pl)
                elif s > us - cs:
                    st = (rs, us, ps)
                else:
                    uu = 2.0 / (g + 1.0) * (cl + (g - 1.0) / 2.0 * ul + s)
                    cc = 2.0 / (g + 1.0) * (cl + (g - 1.0) / 2.0 * (ul - s))
                    rr_ = rl * (cc / cl) ** (2.0 / (g - 1.0))
                    st = (rr_, uu, pl * (cc / cl) ** (2.0 * g / (g - 1.0)))
        else:
            if ps > pr:
                rs = rr * ((ps / pr + gm) / (gm * ps / pr + 1.0))
                sr = ur + cr * math.sqrt((g + 1.0) / (2 * g) * ps / pr + (g - 1.0) / (2 * g))
                st = (rr, ur, pr) if s > sr else (rs, us, ps)
            else:
                rs = rr * (ps / pr) ** (1.0 / g)
                cs = cr * (ps / pr) ** ((g - 1.0) / (2 * g))
                if s > ur + cr:
                    st = (rr, ur, pr)
                elif s < us + cs:
                    st = (rs, us, ps)
                else:
                    uu = 2.0 / (g + 1.0) * (-cr + (g - 1.0) / 2.0 * ur + s)
                    cc = 2.0 / (g + 1.0) * (cr - (g - 1.0) / 2.0 * (ur - s))
                    rr_ = rr * (cc / cr) ** (2.0 / (g - 1.0))
                    st = (rr_, uu, pr * (cc / cr) ** (2.0 * g / (g - 1.0)))
        rho[n], u[n], p[n] = st
    return rho, u, p


def cell_average(x_lo, h, t, rl, ul, pl, rr, ur, pr, g, sub=64):
    """Cell averages of rho over cells [x_lo + i h, x_lo + (i+1) h] at time t
    (interface at x = 0), by midpoint sub-sampling."""
    off = (np.arange(sub) + 0.5) / sub
    n = len(x_lo)
    xs = (np.asarray(x_lo)[:, None] + h * off[None, :]).reshape(-1)
    rho, u, p = sample(xs / t, rl, ul, pl, rr, ur, pr, g)
    return rho.reshape(n, sub).mean(axis=1)
