"""Exact solution of the one-dimensional Riemann problem for an ideal gas.

Test infrastructure: the textbook construction (pressure function of the
two non-linear waves, Newton iteration for the star pressure, then sampling
the self-similar solution), written independently of the oracle.
"""
import math

import numpy as np


def _f(p, rho, pk, ck, g):
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        q = math.sqrt(A / (p + B))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (p + B))
    r = p / pk  # rarefaction
    f = 2.0 * ck / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0)
    return f, 1.0 / (rho * ck) * r ** (-(g + 1.0) / (2.0 * g))


def star_state(L, R, g=1.4):
    """L, R = (rho, u, p). Returns (p*, u*, rho*L, rho*R)."""
    rl, ul, pl = L
    rr, ur, pr = R
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    p = max(1e-12, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dl = _f(p, rl, pl, cl, g)
        fr, dr = _f(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dl + dr)
        pn = max(1e-14, p - dp)
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f(p, rl, pl, cl, g)
    fr, _ = _f(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)

    def rho_star(rk, pk):
        if p > pk:
            q = (g - 1.0) / (g + 1.0)
            return rk * (p / pk + q) / (q * p / pk + 1.0)
        return rk * (p / pk) ** (1.0 / g)

    return p, u, rho_star(rl, pl), rho_star(rr, pr)


def sample(x, t, L, R, x0=0.5, g=1.4):
    """Density, velocity, pressure at positions x (array) and time t > 0."""
    rl, ul, pl = L
    rr, ur, pr = R
    ps, us, rsl, rsr = star_state(L, R, g)
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    out = np.zeros((3, len(x)))
    for n, xx in enumerate(x):
        s = (xx - x0) / t
        if s <= us:  # left of contact
            if ps > pl:
                sl = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                st = (rl, ul, pl) if s <= sl else (rsl, us, ps)
            else:
                csl = cl * (ps / pl) ** ((g - 1) / (2 * g))
                head, tail = ul - cl, us - csl
                if s <= head:
                    st = (rl, ul, pl)
                elif s >= tail:
                    st = (rsl, us, ps)
                else:
                    u = 2.0 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    c = 2.0 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    r = rl * (c / cl) ** (2 / (g - 1))
                    st = (r, u, pl * (c / cl) ** (2 * g / (g - 1)))
        else:
            if ps > pr:
                sr = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                st = (rr, ur, pr) if s >= sr else (rsr, us, ps)
            else:
                csr = cr * (ps / pr) ** ((g - 1) / (2 * g))
                head, tail = ur + cr, us + csr
                if s >= head:
                    st = (rr, ur, pr)
                elif s <= tail:
                    st = (rsr, us, ps)
                else:
                    u = 2.0 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    c = 2.0 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    r = rr * (c / cr) ** (2 / (g - 1))
                    st = (r, u, pr * (c / cr) ** (2 * g / (g - 1)))
        out[:, n] = st
    return out
