"""Exact solution of the 1-D Euler Riemann problem (ideal gas), the textbook
construction: Newton iteration on the pressure function for the star state,
then sampling of the self-similar solution.  Used to pin the oracle on the Sod
shock tube (Sec. 5.2 (b))."""
import math

import numpy as np


def _fk(p, rho, pk, gamma):
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


def star_state(L, R, gamma=1.4):
    rl, ul, pl = L
    rr, ur, pr = R
    p = 0.5 * (pl + pr)
    for _ in range(100):
        fl, dfl = _fk(p, rl, pl, gamma)
        fr, dfr = _fk(p, rr, pr, gamma)
        pn = p - (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(pn, 1e-14)
        if abs(pn - p) < 1e-15 * p:
            p = pn
            break
        p = pn
    fl, _ = _fk(p, rl, pl, gamma)
    fr, _ = _fk(p, rr, pr, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(L, R, s, gamma=1.4):
    """(rho, u, p) at similarity coordinate s = (x - x0)/t."""
    rl, ul, pl = L
    rr, ur, pr = R
    ps, us = star_state(L, R, gamma)
    g = gamma
    if s <= us:
        al = math.sqrt(g * pl / rl)
        if ps > pl:
            sl = ul - al * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
            if s <= sl:
                return rl, ul, pl
            return rl * (ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1), us, ps
        shl = ul - al
        if s <= shl:
            return rl, ul, pl
        asl = al * (ps / pl) ** ((g - 1) / (2 * g))
        stl = us - asl
        if s > stl:
            return rl * (ps / pl) ** (1 / g), us, ps
        u = 2 / (g + 1) * (al + (g - 1) / 2 * ul + s)
        c = 2 / (g + 1) * (al + (g - 1) / 2 * (ul - s))
        rho = rl * (c / al) ** (2 / (g - 1))
        return rho, u, pl * (c / al) ** (2 * g / (g - 1))
    ar = math.sqrt(g * pr / rr)
    if ps > pr:
        sr = ur + ar * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
        if s >= sr:
            return rr, ur, pr
        return rr * (ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1), us, ps
    shr = ur + ar
    if s >= shr:
        return rr, ur, pr
    asr = ar * (ps / pr) ** ((g - 1) / (2 * g))
    str_ = us + asr
    if s < str_:
        return rr * (ps / pr) ** (1 / g), us, ps
    u = 2 / (g + 1) * (-ar + (g - 1) / 2 * ur + s)
    c = 2 / (g + 1) * (ar - (g - 1) / 2 * (ur - s))
    rho = rr * (c / ar) ** (2 / (g - 1))
    return rho, u, pr * (c / ar) ** (2 * g / (g - 1))


def cell_average_density(L, R, n, t, x0=0.5, sub=64, gamma=1.4):
    """Cell averages of the exact density on n cells of [0, 1] (midpoint rule
    with `sub` points per cell)."""
    dx = 1.0 / n
    xs = (np.arange(n * sub) + 0.5) * dx / sub
    rho = np.array([sample(L, R, (x - x0) / t, gamma)[0] for x in xs])
    return rho.reshape(n, sub).mean(axis=1)
