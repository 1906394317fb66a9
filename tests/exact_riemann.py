"""Exact solutions of the Riemann problem of the 1D Euler equations, for an ideal gas and
for an isothermal gas.

Textbook construction: the star pressure (density, isothermal) is the root of
f_L + f_R + (u_R - u_L) = 0 with the shock (Rankine-Hugoniot) and rarefaction branches of
f_K, solved by Newton iteration; the solution is then sampled along x/t.  Used only to
pin the CPU oracle on shock tubes.
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


# ---------------------------------------------------------------------------------
# isothermal gas (p = c^2 rho)
# ---------------------------------------------------------------------------------
#
# Across a shock that connects state K to a star density r the mass flux through the
# shock is c sqrt(rho_K r) (from the mass and momentum jump conditions with p = c^2 rho),
# so the velocity changes by c (r - rho_K)/sqrt(rho_K r); across a rarefaction the
# Riemann invariant u +- c ln(rho) is constant, so it changes by c ln(r/rho_K).  The star
# density is the root of f_L(r) + f_R(r) + (u_R - u_L) = 0.

def _fK_iso(r, rk, c):
    if r > rk:  # shock
        s = math.sqrt(rk * r)
        return c * (r - rk) / s, c * (0.5 / s + 0.5 * rk / (r * s))
    return c * math.log(r / rk), c / r


def iso_star_state(rl, ul, rr, ur, c):
    r = math.sqrt(rl * rr)
    for _ in range(200):
        fl, dfl = _fK_iso(r, rl, c)
        fr, dfr = _fK_iso(r, rr, c)
        dr = (fl + fr + ur - ul) / (dfl + dfr)
        r = max(r - dr, 1e-14)
        if abs(dr) < 1e-15 * r:
            break
    fl, _ = _fK_iso(r, rl, c)
    fr, _ = _fK_iso(r, rr, c)
    return r, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def iso_sample(xi, rl, ul, rr, ur, c):
    """(rho, u) of the isothermal Riemann problem at xi = x/t."""
    rs, us = iso_star_state(rl, ul, rr, ur, c)
    out = np.zeros((2, len(xi)))
    for n, s in enumerate(xi):
        if s <= us:
            if rs > rl:  # left shock, speed u_L - c sqrt(r*/rho_L)
                out[:, n] = (rl, ul) if s <= ul - c * math.sqrt(rs / rl) else (rs, us)
            elif s <= ul - c:
                out[:, n] = (rl, ul)
            elif s >= us - c:
                out[:, n] = (rs, us)
            else:  # inside the left fan: u - c = xi, u + c ln rho = u_L + c ln rho_L
                out[:, n] = (rl * math.exp((ul - s) / c - 1.0), s + c)
        else:
            if rs > rr:  # right shock, speed u_R + c sqrt(r*/rho_R)
                out[:, n] = (rr, ur) if s >= ur + c * math.sqrt(rs / rr) else (rs, us)
            elif s >= ur + c:
                out[:, n] = (rr, ur)
            elif s <= us + c:
                out[:, n] = (rs, us)
            else:  # inside the right fan: u + c = xi, u - c ln rho = u_R - c ln rho_R
                out[:, n] = (rr * math.exp((s - ur) / c - 1.0), s - c)
    return out


def iso_cell_averages(x_edges, t, x0, left, right, c, sub=64):
    n = len(x_edges) - 1
    avg = np.zeros((2, n))
    for i in range(n):
        xs = np.linspace(x_edges[i], x_edges[i + 1], sub + 1)
        xm = 0.5 * (xs[1:] + xs[:-1])
        avg[:, i] = iso_sample((xm - x0) / t, *left, *right, c).mean(axis=1)
    return avg
