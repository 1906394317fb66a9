"""Exact solution of the Riemann problem of the 1D Euler equations (ideal gas).

Textbook construction: the star pressure is the root of f_L(p) + f_R(p) + (u_R - u_L) = 0
with the shock (Rankine-Hugoniot) and rarefaction (isentropic) branches of f_K, solved by
Newton iteration; the solution is then sampled along x/t.  Used only to pin the CPU
oracle on Sod's shock tube.
"""
import math

import numpy as np


def _fK(p, rho, pk, gamma):
    a = math.sqrt(gamma * pk / rho)
    if p > pk:  # shock
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        f = (p - pk) * math.sqrt(A / (p + B))
        df = math.sqrt(A / (B + p)) * (1.0 - 0.5 * (p - pk) / (B + p))
    else:  # rarefaction
        f = 2.0 * a / (gamma - 1.0) * ((p / pk) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)
        df = 1.0 / (rho * a) * (p / pk) ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def star_state(rl, ul, pl, rr, ur, pr, gamma):
    p = 0.5 * (pl + pr)
    for _ in range(100):
        fl, dfl = _fK(p, rl, pl, gamma)
        fr, dfr = _fK(p, rr, pr, gamma)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        p = max(p - dp, 1e-14)
        if abs(dp) < 1e-15 * p:
            break
    fl, _ = _fK(p, rl, pl, gamma)
    fr, _ = _fK(p, rr, pr, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(xi, rl, ul, pl, rr, ur, pr, gamma):
    """(rho, u, p) at similarity coordinate xi = x/t."""
    ps, us = star_state(rl, ul, pl, rr, ur, pr, gamma)
    g = gamma
    out = np.zeros((3, len(xi)))
    al = math.sqrt(g * pl / rl)
    ar = math.sqrt(g * pr / rr)
    for n, s in enumerate(xi):
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                sl = ul - al * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if s <= sl:
                    out[:, n] = (rl, ul, pl)
                else:
                    r = rl * ((ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1))
                    out[:, n] = (r, us, ps)
            else:  # left rarefaction
                shl = ul - al
                asl = al * (ps / pl) ** ((g - 1) / (2 * g))
                stl = us - asl
                if s <= shl:
                    out[:, n] = (rl, ul, pl)
                elif s >= stl:
                    out[:, n] = (rl * (ps / pl) ** (1 / g), us, ps)
                else:
                    u = 2 / (g + 1) * (al + (g - 1) / 2 * ul + s)
                    c = 2 / (g + 1) * (al + (g - 1) / 2 * (ul - s))
                    r = rl * (c / al) ** (2 / (g - 1))
                    out[:, n] = (r, u, pl * (c / al) ** (2 * g / (g - 1)))
        else:  # right of contact
            if ps > pr:  # right shock
                sr = ur + ar * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                if s >= sr:
                    out[:, n] = (rr, ur, pr)
                else:
                    r = rr * ((ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1))
                    out[:, n] = (r, us, ps)
            else:
                shr = ur + ar
                asr = ar * (ps / pr) ** ((g - 1) / (2 * g))
                stvolume = us + asr
                if s >= shr:
                    out[:, n] = (rr, ur, pr)
                elif s <= stvolume:
                    out[:, n] = (rr * (ps / pr) ** (1 / g), us, ps)
                else:
                    u = 2 / (g + 1) * (-ar + (g - 1) / 2 * ur + s)
                    c = 2 / (g + 1) * (ar - (g - 1) / 2 * (ur - s))
                    r = rr * (c / ar) ** (2 / (g - 1))
                    out[:, n] = (r, u, pr * (c / ar) ** (2 * g / (g - 1)))
    return out


def cell_averages(x_edges, t, x0, left, right, gamma, sub=64):
    """Cell averages of the exact solution over cells [x_edges[i], x_edges[i+1]]."""
    n = len(x_edges) - 1
    avg = np.zeros((3, n))
    for i in range(n):
        xs = np.linspace(x_edges[i], x_edges[i + 1], sub + 1)
        xm = 0.5 * (xs[1:] + xs[:-1])
        v = sample((xm - x0) / t, *left, *right, gamma)
        avg[:, i] = v.mean(axis=1)
    return avg
