"""Exact solution of the 1D Euler Riemann problem (ideal gas).

TEST INFRASTRUCTURE ONLY.  The paper's schemes are built on local Riemann
problems (Sec. 1.1, citing Toro's textbook); the exact solver below follows
that textbook's construction (pressure function, Newton iteration for the
star pressure, sampling of the self-similar solution) and pins the oracle's
whole scheme on the Sod tube.  It shares nothing with the oracle or the HIP
path.
"""
from __future__ import annotations

import math

import numpy as np


def _f(p, rho, pk, ck, g):
    """Pressure function of one side and its derivative."""
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        q = math.sqrt(A / (p + B))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (B + p))
    # rarefaction
    r = p / pk
    e = (g - 1.0) / (2.0 * g)
    return 2.0 * ck / (g - 1.0) * (r ** e - 1.0), 1.0 / (rho * ck) * r ** (-(g + 1.0) / (2.0 * g))


def star_state(rl, ul, pl, rr, ur, pr, g=1.4, tol=1e-15):
    """(p*, u*) by Newton iteration on f_L(p) + f_R(p) + u_R - u_L = 0."""
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    p = max(tol, 0.5 * (pl + pr))
    for _ in range(200):
        fl, dl = _f(p, rl, pl, cl, g)
        fr, dr = _f(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dl + dr)
        pn = max(tol, p - dp)
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f(p, rl, pl, cl, g)
    fr, _ = _f(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(xi, rl, ul, pl, rr, ur, pr, g=1.4):
    """(rho, u, p) at similarity coordinate xi = (x - x0) / t."""
    p_s, u_s = star_state(rl, ul, pl, rr, ur, pr, g)
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    gm = (g - 1.0) / (g + 1.0)
    if xi <= u_s:  # left of contact
        if p_s > pl:
            sl = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * p_s / pl + (g - 1.0) / (2.0 * g))
            if xi <= sl:
                return rl, ul, pl
            return rl * ((p_s / pl + gm) / (gm * p_s / pl + 1.0)), u_s, p_s
        shl = ul - cl
        if xi <= shl:
            return rl, ul, pl
        cs = cl * (p_s / pl) ** ((g - 1.0) / (2.0 * g))
        stl = u_s - cs
        if xi > stl:
            return rl * (p_s / pl) ** (1.0 / g), u_s, p_s
        u = 2.0 / (g + 1.0) * (cl + (g - 1.0) / 2.0 * ul + xi)
        c = 2.0 / (g + 1.0) * (cl + (g - 1.0) / 2.0 * (ul - xi))
        rho = rl * (c / cl) ** (2.0 / (g - 1.0))
        return rho, u, pl * (c / cl) ** (2.0 * g / (g - 1.0))
    if p_s > pr:
        sr = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * p_s / pr + (g - 1.0) / (2.0 * g))
        if xi >= sr:
            return rr, ur, pr
        return rr * ((p_s / pr + gm) / (gm * p_s / pr + 1.0)), u_s, p_s
    shr = ur + cr
    if xi >= shr:
        return rr, ur, pr
    cs = cr * (p_s / pr) ** ((g - 1.0) / (2.0 * g))
    str_ = u_s + cs
    if xi <= str_:
        return rr * (p_s / pr) ** (1.0 / g), u_s, p_s
    u = 2.0 / (g + 1.0) * (-cr + (g - 1.0) / 2.0 * ur + xi)
    c = 2.0 / (g + 1.0) * (cr - (g - 1.0) / 2.0 * (ur - xi))
    rho = rr * (c / cr) ** (2.0 / (g - 1.0))
    return rho, u, pr * (c / cr) ** (2.0 * g / (g - 1.0))


def sod_profile(x: np.ndarray, t: float, x0=0.5, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1), g=1.4):
    """Exact (rho, u, p) of the Sod tube at positions x and time t > 0."""
    out = np.empty((3, len(x)))
    for i, xv in enumerate(x):
        out[:, i] = sample((xv - x0) / t, *left, *right, g=g)
    return out


def wave_positions(t: float, x0=0.5, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1), g=1.4):
    """Rarefaction head/tail, contact and shock positions of the Sod tube."""
    rl, ul, pl = left
    rr, ur, pr = right
    p_s, u_s = star_state(rl, ul, pl, rr, ur, pr, g)
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    cs = cl * (p_s / pl) ** ((g - 1.0) / (2.0 * g))
    sr = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * p_s / pr + (g - 1.0) / (2.0 * g))
    return {
        "head": x0 + (ul - cl) * t,
        "tail": x0 + (u_s - cs) * t,
        "contact": x0 + u_s * t,
        "shock": x0 + sr * t,
    }


# ---------------------------------------------------------------------------
# polytrope p = c_ad rho^gamma without energy equation (the shallow water
# equations for rho = h, c_ad = 1/2, gamma = 2): two-wave Riemann problem.
# Each wave is a rarefaction (Riemann invariant u +- 2c/(gamma-1)) or a shock
# (mass and momentum jump conditions only); the star density solves
# f_L(rho) + f_R(rho) + u_R - u_L = 0 with f_K increasing in rho.
# ---------------------------------------------------------------------------


def _poly_p(rho, g, cad):
    return cad * rho ** g


def _poly_c(rho, g, cad):
    return math.sqrt(g * cad * rho ** (g - 1.0))


def _poly_f(rho, rk, g, cad):
    if rho > rk:  # shock: |u* - u_K| = sqrt((p - p_K)(rho - rho_K) / (rho rho_K))
        return math.sqrt((_poly_p(rho, g, cad) - _poly_p(rk, g, cad)) * (rho - rk) / (rho * rk))
    if g == 1.0:  # isothermal rarefaction
        return _poly_c(rk, g, cad) * math.log(rho / rk)
    return 2.0 / (g - 1.0) * (_poly_c(rho, g, cad) - _poly_c(rk, g, cad))


def poly_star(rl, ul, rr, ur, g=2.0, cad=0.5):
    """(rho*, u*) by bisection on the monotone star function."""
    F = lambda r: _poly_f(r, rl, g, cad) + _poly_f(r, rr, g, cad) + ur - ul
    lo, hi = 1e-300, max(rl, rr)
    while F(hi) < 0.0:
        hi *= 2.0
    for _ in range(2000):
        mid = 0.5 * (lo + hi)
        if F(mid) < 0.0:
            lo = mid
        else:
            hi = mid
        if hi - lo <= 1e-15 * hi:
            break
    rs = 0.5 * (lo + hi)
    us = 0.5 * (ul + ur) + 0.5 * (_poly_f(rs, rr, g, cad) - _poly_f(rs, rl, g, cad))
    return rs, us


def _poly_side(xi, rk, uk, rs, us, g, cad, sgn):
    """State at xi = x/t on the side of the wave with sign sgn (-1 left, +1
    right), or None when xi lies beyond that wave (in the star region)."""
    ck = _poly_c(rk, g, cad)
    if rs > rk:  # shock: mass flux m = rho_K (u_K - S) = rho* (u* - S)
        m = math.sqrt((_poly_p(rs, g, cad) - _poly_p(rk, g, cad)) * rs * rk / (rs - rk))
        s = uk + sgn * m / rk
        return (rk, uk) if sgn * (xi - s) > 0.0 else None
    head = uk + sgn * ck
    tail = us + sgn * _poly_c(rs, g, cad)
    if sgn * (xi - head) > 0.0:
        return (rk, uk)
    if sgn * (xi - tail) >= 0.0:  # inside the fan: xi = u + sgn c on the invariant
        if g == 1.0:
            c = ck
            u = xi - sgn * c
            return (rk * math.exp(sgn * (u - uk) / c), u)
        c = (g - 1.0) / (g + 1.0) * (sgn * (xi - uk) + 2.0 * ck / (g - 1.0))
        u = xi - sgn * c
        return ((c * c / (g * cad)) ** (1.0 / (g - 1.0)), u)
    return None


def poly_sample(xi, rl, ul, rr, ur, g=2.0, cad=0.5):
    rs, us = poly_star(rl, ul, rr, ur, g, cad)
    side = _poly_side(xi, rl, ul, rs, us, g, cad, -1.0) if xi <= us else _poly_side(xi, rr, ur, rs, us, g, cad, 1.0)
    return side if side is not None else (rs, us)


def poly_profile(x: np.ndarray, t: float, x0: float, left, right, g=2.0, cad=0.5):
    """(rho, u) of the polytrope's Riemann problem at the points x."""
    out = np.array([poly_sample((xx - x0) / t, left[0], left[1], right[0], right[1], g, cad) for xx in x])
    return out[:, 0], out[:, 1]
