"""Exact solution of the 1-D Riemann problem for an ideal gas (Toro, "Riemann
Solvers and Numerical Methods for Fluid Dynamics", Ch. 4): pressure
function, Newton iteration for p*, and sampling of the self-similar solution.
Test helper only."""
import math

import numpy as np


def _fk(p, rho, pk, ck, g):
    if p > pk:   # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        s = math.sqrt(A / (p + B))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (p + B))
    pr = p / pk   # rarefaction
    f = 2.0 * ck / (g - 1.0) * (pr ** ((g - 1.0) / (2.0 * g)) - 1.0)
    df = 1.0 / (rho * ck) * pr ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(L, R, g=1.4):
    rl, ul, pl = L
    rr, ur, pr = R
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    if 2.0 * (cl + cr) / (g - 1.0) <= ur - ul:
        raise ValueError("vacuum generated")
    p = max(1e-12, 0.5 * (pl + pr))
    for _ in range(200):
        fl, dfl = _fk(p, rl, pl, cl, g)
        fr, dfr = _fk(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(1e-14, p - dp)
        if abs(pn - p) < 1e-14 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _fk(p, rl, pl, cl, g)
    fr, _ = _fk(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(L, R, xi, g=1.4):
    """(rho, u, p) at x/t = xi."""
    rl, ul, pl = L
    rr, ur, pr = R
    ps, us = star_state(L, R, g)
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    gm = (g - 1.0) / (g + 1.0)
    if xi <= us:
        if ps > pl:
            S = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
            if xi <= S:
                return rl, ul, pl
            return rl * (ps / pl + gm) / (gm * ps / pl + 1), us, ps
        csl = cl * (ps / pl) ** ((g - 1) / (2 * g))
        if xi <= ul - cl:
            return rl, ul, pl
        if xi > us - csl:
            return rl * (ps / pl) ** (1 / g), us, ps
        c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - xi))
        u = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + xi)
        rho = rl * (c / cl) ** (2 / (g - 1))
        return rho, u, pl * (c / cl) ** (2 * g / (g - 1))
    if ps > pr:
        S = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
        if xi >= S:
            return rr, ur, pr
        return rr * (ps / pr + gm) / (gm * ps / pr + 1), us, ps
    csr = cr * (ps / pr) ** ((g - 1) / (2 * g))
    if xi >= ur + cr:
        return rr, ur, pr
    if xi < us + csr:
        return rr * (ps / pr) ** (1 / g), us, ps
    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - xi))
    u = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + xi)
    rho = rr * (c / cr) ** (2 / (g - 1))
    return rho, u, pr * (c / cr) ** (2 * g / (g - 1))


def bounds(L, R, g=1.4, n=4001, span=10.0):
    """Min and max of rho and p over the whole self-similar solution."""
    vals = np.array([sample(L, R, x, g) for x in np.linspace(-span, span, n)])
    return vals[:, 0].min(), vals[:, 0].max(), vals[:, 2].min(), vals[:, 2].max()


def wave_extent(L, R, g=1.4, n=20001, span=20.0):
    """Largest |x/t| at which the solution differs from the initial states."""
    xs = np.linspace(-span, span, n)
    vals = np.array([sample(L, R, x, g) for x in xs])
    moved = ~(np.all(np.isclose(vals, L), axis=1) | np.all(np.isclose(vals, R), axis=1))
    return np.abs(xs[moved]).max() + 2 * span / n
