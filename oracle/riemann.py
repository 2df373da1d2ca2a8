"""Exact solution of the 1-D Riemann problem for an ideal gas (textbook closed form).

Test infrastructure: pins the thermal step against the exact solution of a
shock tube.  Two-dimensional monatomic gas: gamma = 2 (c_s = sqrt(gamma T), the
compressible-flow section of the paper), p = rho T.

The star-region pressure solves f_L(p) + f_R(p) + (u_R - u_L) = 0 with the
shock / rarefaction branch functions of the Euler equations (Godunov's exact
solver as presented in standard texts, e.g. Toro, "Riemann Solvers and
Numerical Methods for Fluid Dynamics", ch. 4); the solution is then sampled
along x / t.
"""
import math

import numpy as np
from scipy.optimize import brentq


def _branch(p, rho_k, p_k, gamma):
    a_k = math.sqrt(gamma * p_k / rho_k)
    if p > p_k:  # shock
        A = 2.0 / ((gamma + 1.0) * rho_k)
        B = (gamma - 1.0) / (gamma + 1.0) * p_k
        return (p - p_k) * math.sqrt(A / (p + B))
    # rarefaction
    return 2.0 * a_k / (gamma - 1.0) * ((p / p_k) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)


def star_state(left, right, gamma=2.0):
    """left/right = (rho, u, p).  Returns (p_star, u_star)."""
    rl, ul, pl = left
    rr, ur, pr = right
    fun = lambda p: _branch(p, rl, pl, gamma) + _branch(p, rr, pr, gamma) + (ur - ul)
    lo, hi = 1e-12, 10.0 * max(pl, pr)
    while fun(hi) < 0:
        hi *= 2.0
    p_star = brentq(fun, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
    u_star = 0.5 * (ul + ur) + 0.5 * (_branch(p_star, rr, pr, gamma) - _branch(p_star, rl, pl, gamma))
    return p_star, u_star


def sample(left, right, xi, gamma=2.0):
    """Exact (rho, u, p) at similarity coordinates xi = (x - x_d) / t (array)."""
    rl, ul, pl = left
    rr, ur, pr = right
    p_s, u_s = star_state(left, right, gamma)
    g = gamma
    al = math.sqrt(g * pl / rl)
    ar = math.sqrt(g * pr / rr)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    gm = (g - 1.0) / (g + 1.0)
    for k, s in enumerate(xi.ravel()):
        if s <= u_s:  # left of the contact
            if p_s > pl:  # left shock
                sl = ul - al * math.sqrt((g + 1) / (2 * g) * p_s / pl + (g - 1) / (2 * g))
                if s <= sl:
                    r, uu, pp = rl, ul, pl
                else:
                    r = rl * ((p_s / pl + gm) / (gm * p_s / pl + 1.0))
                    uu, pp = u_s, p_s
            else:  # left rarefaction
                a_s = al * (p_s / pl) ** ((g - 1) / (2 * g))
                head, tail = ul - al, u_s - a_s
                if s <= head:
                    r, uu, pp = rl, ul, pl
                elif s >= tail:
                    r, uu, pp = rl * (p_s / pl) ** (1.0 / g), u_s, p_s
                else:
                    c = 2.0 / (g + 1) + (g - 1) / ((g + 1) * al) * (ul - s)
                    r = rl * c ** (2.0 / (g - 1))
                    uu = 2.0 / (g + 1) * (al + (g - 1) / 2 * ul + s)
                    pp = pl * c ** (2 * g / (g - 1))
        else:  # right of the contact
            if p_s > pr:  # right shock
                sr = ur + ar * math.sqrt((g + 1) / (2 * g) * p_s / pr + (g - 1) / (2 * g))
                if s >= sr:
                    r, uu, pp = rr, ur, pr
                else:
                    r = rr * ((p_s / pr + gm) / (gm * p_s / pr + 1.0))
                    uu, pp = u_s, p_s
            else:  # right rarefaction
                a_s = ar * (p_s / pr) ** ((g - 1) / (2 * g))
                head, tail = ur + ar, u_s + a_s
                if s >= head:
                    r, uu, pp = rr, ur, pr
                elif s <= tail:
                    r, uu, pp = rr * (p_s / pr) ** (1.0 / g), u_s, p_s
                else:
                    c = 2.0 / (g + 1) - (g - 1) / ((g + 1) * ar) * (ur - s)
                    r = rr * c ** (2.0 / (g - 1))
                    uu = 2.0 / (g + 1) * (-ar + (g - 1) / 2 * ur + s)
                    pp = pr * c ** (2 * g / (g - 1))
        rho.flat[k], u.flat[k], p.flat[k] = r, uu, pp
    return rho, u, p


def wave_speeds(left, right, gamma=2.0):
    """(rarefaction head, rarefaction tail, contact, shock) speeds of the Sod-type problem."""
    rl, ul, pl = left
    rr, ur, pr = right
    p_s, u_s = star_state(left, right, gamma)
    g = gamma
    al = math.sqrt(g * pl / rl)
    ar = math.sqrt(g * pr / rr)
    a_s = al * (p_s / pl) ** ((g - 1) / (2 * g))
    shock = ur + ar * math.sqrt((g + 1) / (2 * g) * p_s / pr + (g - 1) / (2 * g))
    return ul - al, u_s - a_s, u_s, shock
