"""Exact solution of the 1D Riemann problem for the ideal-gas Euler equations
(Toro, "Riemann Solvers and Numerical Methods for Fluid Dynamics", 3rd ed.,
2009, ch. 4): Newton iteration on the pressure function f(p) = f_L + f_R + du,
then sampling of the self-similar solution.  Used only to pin the oracle."""
import math

import numpy as np


def _fk(p, rk, pk, ck, g):
    if p > pk:  # shock
        A = 2.0 / ((g + 1) * rk)
        B = (g - 1) / (g + 1) * pk
        q = math.sqrt(A / (p + B))
        return (p - pk) * q, q * (1 - 0.5 * (p - pk) / (B + p))
    pr = p / pk  # rarefaction
    f = 2 * ck / (g - 1) * (pr ** ((g - 1) / (2 * g)) - 1)
    return f, 1.0 / (rk * ck) * pr ** (-(g + 1) / (2 * g))


def star_state(rl, ul, pl, rr, ur, pr, g=1.4):
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    p = max(1e-8, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dl = _fk(p, rl, pl, cl, g)
        fr, dr = _fk(p, rr, pr, cr, g)
        pn = max(1e-12, p - (fl + fr + ur - ul) / (dl + dr))
        if abs(pn - p) < 1e-14 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _fk(p, rl, pl, cl, g)
    fr, _ = _fk(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(xi, rl, ul, pl, rr, ur, pr, g=1.4):
    """(rho, u, p) at x/t = xi (arrays)."""
    ps, us = star_state(rl, ul, pl, rr, ur, pr, g)
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi); u = np.empty_like(xi); p = np.empty_like(xi)
    gm = (g - 1) / (g + 1)
    for n, s in enumerate(xi.ravel()):
        if s <= us:  # left of contact
            if ps > pl:
                sl = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if s <= sl:
                    r, v, q = rl, ul, pl
                else:
                    r, v, q = rl * (ps / pl + gm) / (gm * ps / pl + 1), us, ps
            else:
                shl = ul - cl
                csl = cl * (ps / pl) ** ((g - 1) / (2 * g))
                stl = us - csl
                if s <= shl:
                    r, v, q = rl, ul, pl
                elif s >= stl:
                    r, v, q = rl * (ps / pl) ** (1 / g), us, ps
                else:
                    v = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    r = rl * (c / cl) ** (2 / (g - 1))
                    q = pl * (c / cl) ** (2 * g / (g - 1))
        else:
            if ps > pr:
                sr = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                if s >= sr:
                    r, v, q = rr, ur, pr
                else:
                    r, v, q = rr * (ps / pr + gm) / (gm * ps / pr + 1), us, ps
            else:
                shr = ur + cr
                csr = cr * (ps / pr) ** ((g - 1) / (2 * g))
                str_ = us + csr
                if s >= shr:
                    r, v, q = rr, ur, pr
                elif s <= str_:
                    r, v, q = rr * (ps / pr) ** (1 / g), us, ps
                else:
                    v = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    r = rr * (c / cr) ** (2 / (g - 1))
                    q = pr * (c / cr) ** (2 * g / (g - 1))
        rho.flat[n], u.flat[n], p.flat[n] = r, v, q
    return rho, u, p
