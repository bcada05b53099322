"""Exact solution of the Riemann problem for the 1D Euler equations of an
ideal gas (the textbook construction: a star-region pressure from the
shock/rarefaction pressure functions by Newton iteration, then self-similar
sampling).  Test infrastructure: an independent reference for the shock
path at high Reynolds numbers, where the viscous solutions approach it."""

import math

import numpy as np


def _f(p, rho, pk, c, g):
    """Pressure function of one side and its derivative."""
    if p > pk:                                    # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        q = math.sqrt(A / (p + B))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (p + B))
    r = p / pk                                    # rarefaction
    return (2.0 * c / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0),
            r ** (-(g + 1.0) / (2.0 * g)) / (rho * c))


def star_state(left, right, g=1.4):
    """(p*, u*) for primitive states (rho, u, p) on either side."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    if 2.0 * (cl + cr) / (g - 1.0) <= ur - ul:
        raise ValueError('vacuum is generated')
    # two-rarefaction guess, safe for strong pressure ratios
    z = (g - 1.0) / (2.0 * g)
    p = ((cl + cr - 0.5 * (g - 1.0) * (ur - ul)) / (cl / pl ** z + cr / pr ** z)) ** (1.0 / z)
    for _ in range(200):
        fl, dl = _f(p, rl, pl, cl, g)
        fr, dr = _f(p, rr, pr, cr, g)
        step = (fl + fr + ur - ul) / (dl + dr)
        pn = max(p - step, 1e-14 * p)
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f(p, rl, pl, cl, g)
    fr, _ = _f(p, rr, pr, cr, g)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def sample(left, right, xi, g=1.4):
    """Primitive (rho, u, p) at the similarity coordinates xi = (x - x0) / t."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    ps, us = star_state(left, right, g)
    gm = (g - 1.0) / (g + 1.0)
    out = np.zeros((3, len(xi)))
    for n, s in enumerate(np.asarray(xi, dtype=float)):
        if s <= us:                              # left of the contact
            if ps > pl:
                S = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
                w = (rl, ul, pl) if s <= S else (rl * (ps / pl + gm) / (gm * ps / pl + 1.0), us, ps)
            else:
                head, cs = ul - cl, cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))
                tail = us - cs
                if s <= head:
                    w = (rl, ul, pl)
                elif s >= tail:
                    w = (rl * (ps / pl) ** (1.0 / g), us, ps)
                else:
                    k = 2.0 / (g + 1.0) + gm / cl * (ul - s)
                    w = (rl * k ** (2.0 / (g - 1.0)), 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + s),
                         pl * k ** (2.0 * g / (g - 1.0)))
        else:                                    # right of the contact
            if ps > pr:
                S = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
                w = (rr, ur, pr) if s >= S else (rr * (ps / pr + gm) / (gm * ps / pr + 1.0), us, ps)
            else:
                head, cs = ur + cr, cr * (ps / pr) ** ((g - 1.0) / (2.0 * g))
                tail = us + cs
                if s >= head:
                    w = (rr, ur, pr)
                elif s <= tail:
                    w = (rr * (ps / pr) ** (1.0 / g), us, ps)
                else:
                    k = 2.0 / (g + 1.0) - gm / cr * (ur - s)
                    w = (rr * k ** (2.0 / (g - 1.0)), 2.0 / (g + 1.0) * (-cr + 0.5 * (g - 1.0) * ur + s),
                         pr * k ** (2.0 * g / (g - 1.0)))
        out[:, n] = w
    return out


def cell_averages(left, right, x0, x1, xd, t, nx, g=1.4, sub=64):
    """Cell averages of (rho, rho u, E) on nx uniform cells of [x0, x1] at time
    t, by the midpoint rule on ``sub`` points per cell."""
    h = (x1 - x0) / nx
    x = x0 + h * (np.arange(nx * sub) + 0.5) / sub
    r, u, p = sample(left, right, (x - xd) / t, g)
    U = np.stack([r, r * u, p / (g - 1.0) + 0.5 * r * u * u])
    return U.reshape(3, nx, sub).mean(axis=2)
