"""Exact solution of the Riemann problem for the ideal-gas Euler equations.

Independent pin for the oracle: pressure function and Newton iteration for the
star pressure, then sampling of the self-similar solution (Toro, "Riemann
Solvers and Numerical Methods for Fluid Dynamics", 3rd ed. 2009, chapter 4).
Shares no code with the oracle.
"""
from __future__ import annotations

import math

import numpy as np


def _f_and_df(p, rho, pk, ck, gamma):
    if p > pk:  # shock
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        s = math.sqrt(A / (p + B))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (B + p))
    # rarefaction
    r = p / pk
    f = 2.0 * ck / (gamma - 1.0) * (r ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)
    df = 1.0 / (rho * ck) * r ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def star_state(rl, ul, pl, rr, ur, pr, gamma=1.4, tol=1e-15):
    """Star-region pressure and velocity (Newton iteration on f_L + f_R + du = 0)."""
    cl = math.sqrt(gamma * pl / rl)
    cr = math.sqrt(gamma * pr / rr)
    du = ur - ul
    p = max(tol, 0.5 * (pl + pr) - 0.125 * du * (rl + rr) * (cl + cr))
    for _ in range(100):
        fl, dfl = _f_and_df(p, rl, pl, cl, gamma)
        fr, dfr = _f_and_df(p, rr, pr, cr, gamma)
        pn = p - (fl + fr + du) / (dfl + dfr)
        pn = max(pn, tol)
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f_and_df(p, rl, pl, cl, gamma)
    fr, _ = _f_and_df(p, rr, pr, cr, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(xi, rl, ul, pl, rr, ur, pr, gamma=1.4):
    """Solution (rho, u, p) at similarity coordinates xi = (x - x0) / t."""
    ps, us = star_state(rl, ul, pl, rr, ur, pr, gamma)
    cl = math.sqrt(gamma * pl / rl)
    cr = math.sqrt(gamma * pr / rr)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for n, s in enumerate(xi):
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                rsl = rl * ((ps / pl + g1) / (ps / pl * g1 + 1.0))
                sl = ul - cl * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pl + (gamma - 1.0) / (2.0 * gamma))
                rho[n], u[n], p[n] = (rl, ul, pl) if s <= sl else (rsl, us, ps)
            else:  # left rarefaction
                shl = ul - cl
                csl = cl * (ps / pl) ** ((gamma - 1.0) / (2.0 * gamma))
                stl = us - csl
                if s <= shl:
                    rho[n], u[n], p[n] = rl, ul, pl
                elif s >= stl:
                    rho[n], u[n], p[n] = rl * (ps / pl) ** (1.0 / gamma), us, ps
                else:
                    c = 2.0 / (gamma + 1.0) * (cl + 0.5 * (gamma - 1.0) * (ul - s))
                    uu = 2.0 / (gamma + 1.0) * (cl + 0.5 * (gamma - 1.0) * ul + s)
                    rho[n] = rl * (c / cl) ** (2.0 / (gamma - 1.0))
                    u[n] = uu
                    p[n] = pl * (c / cl) ** (2.0 * gamma / (gamma - 1.0))
        else:  # right of contact
            if ps > pr:  # right shock
                rsr = rr * ((ps / pr + g1) / (ps / pr * g1 + 1.0))
                sr = ur + cr * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pr + (gamma - 1.0) / (2.0 * gamma))
                rho[n], u[n], p[n] = (rr, ur, pr) if s >= sr else (rsr, us, ps)
            else:  # right rarefaction
                shr = ur + cr
                csr = cr * (ps / pr) ** ((gamma - 1.0) / (2.0 * gamma))
                stR = us + csr
                if s >= shr:
                    rho[n], u[n], p[n] = rr, ur, pr
                elif s <= stR:
                    rho[n], u[n], p[n] = rr * (ps / pr) ** (1.0 / gamma), us, ps
                else:
                    c = 2.0 / (gamma + 1.0) * (cr - 0.5 * (gamma - 1.0) * (ur - s))
                    uu = 2.0 / (gamma + 1.0) * (-cr + 0.5 * (gamma - 1.0) * ur + s)
                    rho[n] = rr * (c / cr) ** (2.0 / (gamma - 1.0))
                    u[n] = uu
                    p[n] = pr * (c / cr) ** (2.0 * gamma / (gamma - 1.0))
    return rho, u, p


def cell_average(x_lo, x_hi, t, x0, left, right, gamma=1.4, sub=64):
    """Cell averages of the exact solution's conserved density, by sub-sampling."""
    out = np.empty(len(x_lo))
    for n, (a, b) in enumerate(zip(x_lo, x_hi)):
        xs = a + (np.arange(sub) + 0.5) * (b - a) / sub
        rho, _, _ = sample((xs - x0) / t, *left, *right, gamma=gamma)
        out[n] = rho.mean()
    return out
