"""Exact solution of the 1D Riemann problem for an ideal gas -- TEST INFRASTRUCTURE.

Written from the textbook mathematics (the pressure-function formulation): the
star pressure p* solves f_L(p*) + f_R(p*) + (u_R - u_L) = 0, where for side K
    f_K(p) = (p - p_K) sqrt(A_K / (p + B_K)),                 p > p_K  (shock)
    f_K(p) = 2 c_K/(g-1) ((p/p_K)^((g-1)/(2g)) - 1),          p <= p_K (rarefaction)
with A_K = 2/((g+1) rho_K), B_K = (g-1)/(g+1) p_K.  The solution is then sampled
at x/t.  A vacuum right state (rho_R = p_R = 0) is a single rarefaction into
vacuum with front speed u_L + 2 c_L/(g-1).
"""
import math

import numpy as np


def _f(p, rho, pk, ck, g):
    if p > pk:
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        s = math.sqrt(A / (p + B))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (B + p))
    r = p / pk
    f = 2.0 * ck / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0)
    df = 1.0 / (rho * ck) * r ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(left, right, g):
    """(p*, u*) for left/right = (rho, u, p), by Newton iteration."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    # two-rarefaction guess
    z = (g - 1.0) / (2.0 * g)
    p = ((cl + cr - 0.5 * (g - 1.0) * (ur - ul)) / (cl / pl ** z + cr / pr ** z)) ** (1.0 / z)
    p = max(p, 1e-12)
    for _ in range(100):
        fl, dl = _f(p, rl, pl, cl, g)
        fr, dr = _f(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dl + dr)
        pn = max(p - dp, 1e-14)
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f(p, rl, pl, cl, g)
    fr, _ = _f(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def waves(left, right, g):
    """Speeds and star densities of the wave pattern (non-vacuum case)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    ps, us = star_state(left, right, g)
    gm = (g - 1.0) / (g + 1.0)
    out = {"p_star": ps, "u_star": us}
    if ps > pl:
        out["rho_star_L"] = rl * (ps / pl + gm) / (gm * ps / pl + 1.0)
        out["S_L"] = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
    else:
        out["rho_star_L"] = rl * (ps / pl) ** (1.0 / g)
        out["head_L"] = ul - cl
        out["tail_L"] = us - cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))
    if ps > pr:
        out["rho_star_R"] = rr * (ps / pr + gm) / (gm * ps / pr + 1.0)
        out["S_R"] = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
    else:
        out["rho_star_R"] = rr * (ps / pr) ** (1.0 / g)
        out["head_R"] = ur + cr
        out["tail_R"] = us + cr * (ps / pr) ** ((g - 1.0) / (2.0 * g))
    return out


def sample(left, right, g, xi):
    """(rho, u, p) at similarity coordinates xi = (x - x0)/t (array)."""
    xi = np.asarray(xi, dtype=np.float64)
    rl, ul, pl = left
    rr, ur, pr = right
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    cl = math.sqrt(g * pl / rl) if rl > 0 else 0.0
    if rr == 0.0 and pr == 0.0:
        # rarefaction into vacuum
        front = ul + 2.0 * cl / (g - 1.0)
        head = ul - cl
        for n, s in enumerate(xi.flat):
            if s <= head:
                r, v, q = rl, ul, pl
            elif s < front:
                v = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + s)
                c = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * (ul - s))
                r = rl * (c / cl) ** (2.0 / (g - 1.0))
                q = pl * (c / cl) ** (2.0 * g / (g - 1.0))
            else:
                r, v, q = 0.0, 0.0, 0.0
            rho.flat[n], u.flat[n], p.flat[n] = r, v, q
        return rho, u, p
    cr = math.sqrt(g * pr / rr)
    ps, us = star_state(left, right, g)
    gm = (g - 1.0) / (g + 1.0)
    for n, s in enumerate(xi.flat):
        if s <= us:  # left of the contact
            if ps > pl:
                SL = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
                if s <= SL:
                    r, v, q = rl, ul, pl
                else:
                    r, v, q = rl * (ps / pl + gm) / (gm * ps / pl + 1.0), us, ps
            else:
                hd = ul - cl
                tl = us - cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))
                if s <= hd:
                    r, v, q = rl, ul, pl
                elif s >= tl:
                    r, v, q = rl * (ps / pl) ** (1.0 / g), us, ps
                else:
                    v = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + s)
                    c = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * (ul - s))
                    r = rl * (c / cl) ** (2.0 / (g - 1.0))
                    q = pl * (c / cl) ** (2.0 * g / (g - 1.0))
        else:
            if ps > pr:
                SR = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
                if s >= SR:
                    r, v, q = rr, ur, pr
                else:
                    r, v, q = rr * (ps / pr + gm) / (gm * ps / pr + 1.0), us, ps
            else:
                hd = ur + cr
                tl = us + cr * (ps / pr) ** ((g - 1.0) / (2.0 * g))
                if s >= hd:
                    r, v, q = rr, ur, pr
                elif s <= tl:
                    r, v, q = rr * (ps / pr) ** (1.0 / g), us, ps
                else:
                    v = 2.0 / (g + 1.0) * (-cr + 0.5 * (g - 1.0) * ur + s)
                    c = 2.0 / (g + 1.0) * (cr - 0.5 * (g - 1.0) * (ur - s))
                    r = rr * (c / cr) ** (2.0 / (g - 1.0))
                    q = pr * (c / cr) ** (2.0 * g / (g - 1.0))
        rho.flat[n], u.flat[n], p.flat[n] = r, v, q
    return rho, u, p


def cell_average(left, right, g, x_edges, x0, t, sub=64):
    """Cell averages of rho, u, p over [x_edges[i], x_edges[i+1]] by midpoint sub-sampling."""
    x_edges = np.asarray(x_edges, dtype=np.float64)
    n = len(x_edges) - 1
    fr = (np.arange(sub) + 0.5) / sub
    xs = x_edges[:-1, None] + (x_edges[1:, None] - x_edges[:-1, None]) * fr[None, :]
    r, u, p = sample(left, right, g, (xs - x0) / t)
    return r.mean(axis=1), u.mean(axis=1), p.mean(axis=1)
