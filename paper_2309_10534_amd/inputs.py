"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds only input generation: exact or Gauss-Legendre cell averages
of analytic initial conditions and seeded random Riemann states.  It contains
none of the scheme's arithmetic and is shared by the HIP path's callers and by
the CPU oracle's tests.  All fields use the layout [component][z][y][x] with
components (rho, rho U, rho V, rho W, rho E) truncated to D+2, FP64.

Workloads (Sec. 5 of the paper):
  * density_wave_1d / density_wave_2d: smooth advection of a density sine
    wave (Sec. 5.1 and 5.5).
  * sod: Sod shock tube (Sec. 5.2 (b)).
  * quadrant_riemann: four constant quadrant states (Sec. 5.6) with seeded
    random states.
  * taylor_green_3d: Taylor-Green vortex (Navier-Stokes, 3-D).
  * isentropic_vortex_2d: translating isentropic vortex (smooth, periodic).
  * riemann_instances: seeded sets of uneven-size 1-D and 2-D Riemann
    problems for batched runs.
"""
from __future__ import annotations

import numpy as np

GAMMA = 1.4


def conservative(rho, vel, p, gamma=GAMMA):
    """Stack (rho, rho*vel..., p/(gamma-1) + rho|vel|^2/2) into a field."""
    rho = np.asarray(rho, dtype=np.float64)
    vel = [np.broadcast_to(np.asarray(v, dtype=np.float64), rho.shape) for v in vel]
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), rho.shape)
    ke = sum(v * v for v in vel) * rho * 0.5
    return np.stack([rho] + [rho * v for v in vel] + [p / (gamma - 1.0) + ke]).astype(np.float64)


def primitive(W, gamma=GAMMA):
    """(rho, [vel...], p) of a conservative field (for diagnostics in tests)."""
    D = W.shape[0] - 2
    rho = W[0]
    vel = [W[1 + d] / rho for d in range(D)]
    ke = sum(v * v for v in vel) * rho * 0.5
    return rho, vel, (gamma - 1.0) * (W[D + 1] - ke)


def _edges(n, lo, hi):
    return np.linspace(lo, hi, n + 1)


def density_wave_1d(n, t=0.0, gamma=GAMMA, L=2.0):
    """Exact cell averages of rho = 1 + 0.2 sin(pi (x - t)), U = 1, p = 1 on [0, L]."""
    e = _edges(n, 0.0, L)
    dx = L / n
    avg_sin = (np.cos(np.pi * (e[:-1] - t)) - np.cos(np.pi * (e[1:] - t))) / (np.pi * dx)
    rho = 1.0 + 0.2 * avg_sin
    # rho U and rho E are linear in rho since U and p are constant
    return np.stack([rho, rho * 1.0, 1.0 / (gamma - 1.0) + 0.5 * rho]), dx


def density_wave_2d(n, t=0.0, gamma=GAMMA, L=2.0):
    """Exact cell averages of rho = 1 + 0.2 sin(pi (x + y - 2t)), U = V = 1, p = 1."""
    e = _edges(n, 0.0, L)
    dx = L / n
    x0, x1 = e[:-1][None, :], e[1:][None, :]
    y0, y1 = e[:-1][:, None], e[1:][:, None]
    c = 2.0 * t
    s = (-np.sin(np.pi * (x1 + y1 - c)) + np.sin(np.pi * (x1 + y0 - c))
         + np.sin(np.pi * (x0 + y1 - c)) - np.sin(np.pi * (x0 + y0 - c))) / (np.pi ** 2 * dx * dx)
    rho = 1.0 + 0.2 * s
    return np.stack([rho, rho, rho, 1.0 / (gamma - 1.0) + rho]), dx


def sod(n=400, gamma=GAMMA):
    """Sod shock tube on [0, 1]: (1, 0, 1) | (0.125, 0, 0.1), split at 0.5."""
    return riemann_1d(n, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), gamma=gamma)


def riemann_1d(n, left, right, x0=0.5, gamma=GAMMA):
    """Area-weighted cell averages of a 1-D Riemann problem on [0, 1]."""
    e = _edges(n, 0.0, 1.0)
    frac_left = np.clip((x0 - e[:-1]) / (e[1:] - e[:-1]), 0.0, 1.0)
    WL = conservative(np.array([left[0]]), [np.array([left[1]])], np.array([left[2]]), gamma)[:, 0]
    WR = conservative(np.array([right[0]]), [np.array([right[1]])], np.array([right[2]]), gamma)[:, 0]
    W = frac_left[None, :] * WL[:, None] + (1.0 - frac_left)[None, :] * WR[:, None]
    return np.ascontiguousarray(W), 1.0 / n


def viscous_shock_tube(nx, ny, gamma=GAMMA):
    """Viscous shock tube (Sec. 5.8): [0, 1] x [0, 1/2], nx x ny cells,
    (rho, U, p) = (120, 0, 120/gamma) for x < 1/2 and (1.2, 0, 1.2/gamma) for
    x > 1/2 (area-weighted across the membrane).  Returns (W [4][ny][nx],
    dx); square cells need ny = nx / 2."""
    W1, dx = riemann_1d(nx, (120.0, 0.0, 120.0 / gamma), (1.2, 0.0, 1.2 / gamma), gamma=gamma)
    W = np.zeros((4, ny, nx))
    W[0] = W1[0][None, :]
    W[1] = W1[1][None, :]
    W[3] = W1[2][None, :]
    return W, dx


def _left_of_line_fraction(x0, x1, y0, y1, a, b):
    """Exact fraction of the cell [x0, x1] x [y0, y1] with x < a + b y
    (b >= 0): the mean over y of clip((a + b y - x0) / (x1 - x0), 0, 1),
    integrated piecewise between the kinks."""
    w = x1 - x0

    def prim(y):  # antiderivative of the unclipped fraction
        return ((a - x0) * y + 0.5 * b * y * y) / w

    if b == 0.0:
        return np.clip((a - x0) / w, 0.0, 1.0) * np.ones_like(y0)
    ya = (x0 - a) / b  # fraction 0 here
    yb = (x1 - a) / b  # fraction 1 here
    lo = np.clip(ya, y0, y1)
    hi = np.clip(yb, y0, y1)
    return ((prim(hi) - prim(lo)) + (y1 - hi)) / (y1 - y0)


DMR_POST = (8.0, 4.125 * np.sqrt(3.0), -4.125, 116.5)
DMR_PRE = (1.4, 0.0, 0.0, 1.0)


def oblique_shock(nx, ny, post, pre, Lx=4.0, Ly=1.0, x0=1.0 / 6.0, gamma=GAMMA):
    """A straight shock at 60 degrees to the x axis through (x0, 0), the line
    x = x0 + y / sqrt 3, with the primitive state post = (rho, U, V, p) on
    its left and pre on its right, on [0, Lx] x [0, Ly]; cells cut by the
    line hold area-weighted averages.  Returns (W [4][ny][nx], (dx, dy), A,
    B) with A, B the conservative states."""
    ex = np.linspace(0.0, Lx, nx + 1)
    ey = np.linspace(0.0, Ly, ny + 1)
    X0, Y0 = np.meshgrid(ex[:-1], ey[:-1])
    X1, Y1 = np.meshgrid(ex[1:], ey[1:])
    f = _left_of_line_fraction(X0, X1, Y0, Y1, x0, 1.0 / np.sqrt(3.0))

    def cons(st):
        return conservative(np.array(st[0]), [np.array(st[1]), np.array(st[2])], np.array(st[3]), gamma)

    A, B = cons(post), cons(pre)
    W = f[None] * A[:, None, None] + (1.0 - f[None]) * B[:, None, None]
    return np.ascontiguousarray(W), (Lx / nx, Ly / ny), A, B


def double_mach(nx=960, ny=240, gamma=GAMMA):
    """Double Mach reflection (Sec. 5.7) on [0, 4] x [0, 1]: a Mach 10 shock
    at 60 degrees to the x axis through (1/6, 0) separates the post-shock
    state (rho, U, V, p) = (8, 4.125 sqrt 3, -4.125, 116.5) (left) from
    (1.4, 0, 0, 1); its line moves as x = 1/6 + (y + 20 t) / sqrt 3.  Returns
    (W [4][ny][nx], (dx, dy), boundary description): the left side takes
    the post-shock state, the right side is transmissive, the bottom takes
    the post-shock state for x < 1/6 and is a slip (reflective) wall beyond,
    the top follows the exact moving shock."""
    W, dxy, A, B = oblique_shock(nx, ny, DMR_POST, DMR_PRE, gamma=gamma)
    s3 = np.sqrt(3.0)
    spec = {
        "bc": [("prescribed", "transmissive"), ("prescribed", "prescribed")],
        "states": (A.tolist(), B.tolist()),
        "lines": {(0, 0): (np.inf, 0.0, 0.0), (1, 0): (1.0 / 6.0, 0.0, 0.0),
                  (1, 1): (1.0 / 6.0, 1.0 / s3, 20.0 / s3)},
        "far": {(1, 0): "reflective", (1, 1): "state_b"},
    }
    return W, dxy, spec


def quadrant_states(rng, rho_range=(0.1, 2.0), vel_range=(-1.0, 1.0), p_range=(0.03, 1.5)):
    """Four (rho, u, v, p) states drawn in quadrant order (x<1/2,y<1/2), (>=,<),
    (>=,>=), (<,>=); rho and p log-uniform, velocities uniform."""
    out = []
    for _ in range(4):
        rho = float(np.exp(rng.uniform(np.log(rho_range[0]), np.log(rho_range[1]))))
        u = float(rng.uniform(*vel_range))
        v = float(rng.uniform(*vel_range))
        p = float(np.exp(rng.uniform(np.log(p_range[0]), np.log(p_range[1]))))
        out.append((rho, u, v, p))
    return out


def quadrant_field(nx, ny, states, x0=0.5, y0=0.5, gamma=GAMMA):
    """Area-weighted cell averages of four constant quadrants on [0,1]^2."""
    ex, ey = _edges(nx, 0.0, 1.0), _edges(ny, 0.0, 1.0)
    fx = np.clip((x0 - ex[:-1]) / np.diff(ex), 0.0, 1.0)  # fraction with x < x0
    fy = np.clip((y0 - ey[:-1]) / np.diff(ey), 0.0, 1.0)
    Wq = [conservative(np.array([s[0]]), [np.array([s[1]]), np.array([s[2]])], np.array([s[3]]), gamma)[:, 0]
          for s in states]
    wts = [np.outer(fy, fx), np.outer(fy, 1 - fx), np.outer(1 - fy, 1 - fx), np.outer(1 - fy, fx)]
    W = sum(w[None] * Wq[k][:, None, None] for k, w in enumerate(wts))
    return np.ascontiguousarray(W)


def quadrant_riemann(n=1024, seed=0, gamma=GAMMA):
    """2-D four-quadrant Riemann problem with seeded states on an n x n grid of [0,1]^2."""
    rng = np.random.default_rng(seed)
    st = quadrant_states(rng)
    return quadrant_field(n, n, st, gamma=gamma), 1.0 / n, st


def _gl(m=4):
    x, w = np.polynomial.legendre.leggauss(m)
    return 0.5 * x, 0.5 * w  # on [-1/2, 1/2], weights sum to 1


def _cell_average(fun, edges, m=4):
    """Gauss-Legendre (m points per axis) cell averages of fun(*coords) -> list of arrays."""
    D = len(edges)
    shape = tuple(len(e) - 1 for e in reversed(edges))  # array order is [z][y][x]
    xg, wg = _gl(m)
    acc = None
    for idx in np.ndindex(*([m] * D)):
        coords = []
        wt = 1.0
        for d in range(D):
            e = edges[d]
            c = 0.5 * (e[:-1] + e[1:]) + xg[idx[d]] * np.diff(e)
            sh = [1] * D
            sh[D - 1 - d] = len(c)
            coords.append(c.reshape(sh))
            wt *= wg[idx[d]]
        vals = [np.broadcast_to(np.asarray(v, dtype=np.float64), shape) for v in fun(*coords)]
        if acc is None:
            acc = [wt * v for v in vals]
        else:
            acc = [a + wt * v for a, v in zip(acc, vals)]
    return np.ascontiguousarray(np.stack(acc))


def isentropic_vortex_2d(n=512, strength=5.0, L=10.0, gamma=GAMMA, m=4, center=None):
    """Isentropic vortex centred at (L/2, L/2) (or `center`) in a mean flow
    (1, 1) on a periodic [0, L]^2; 4x4 Gauss-Legendre cell averages of the
    conservative variables."""
    e = _edges(n, 0.0, L)
    eps = strength
    cx, cy = (0.5 * L, 0.5 * L) if center is None else center

    def fun(x, y):
        xb, yb = x - cx, y - cy
        r2 = xb * xb + yb * yb
        du = eps / (2 * np.pi) * np.exp(0.5 * (1 - r2)) * (-yb)
        dv = eps / (2 * np.pi) * np.exp(0.5 * (1 - r2)) * xb
        dT = -(gamma - 1) * eps * eps / (8 * gamma * np.pi ** 2) * np.exp(1 - r2)
        rho = (1 + dT) ** (1 / (gamma - 1))
        p = rho ** gamma
        u, v = 1 + du, 1 + dv
        return [rho, rho * u, rho * v, p / (gamma - 1) + 0.5 * rho * (u * u + v * v)]

    return _cell_average(fun, [e, e], m), L / n


def taylor_green_3d(n=128, mach=0.1, gamma=GAMMA, m=4):
    """Taylor-Green vortex on a periodic [0, 2 pi]^3 (U0 = rho0 = L = 1):
    u = sin x cos y cos z, v = -cos x sin y cos z, w = 0,
    p = p0 + (cos 2x + cos 2y)(cos 2z + 2)/16, p0 = 1/(gamma Ma^2), rho = p/p0.
    4x4x4 Gauss-Legendre cell averages of the conservative variables."""
    L = 2 * np.pi
    e = _edges(n, 0.0, L)
    p0 = 1.0 / (gamma * mach * mach)

    def fun(x, y, z):
        u = np.sin(x) * np.cos(y) * np.cos(z)
        v = -np.cos(x) * np.sin(y) * np.cos(z)
        w = 0.0 * x * y * z
        p = p0 + (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2) / 16.0
        rho = p / p0
        return [rho, rho * u, rho * v, rho * w, p / (gamma - 1) + 0.5 * rho * (u * u + v * v + w * w)]

    return _cell_average(fun, [e, e, e], m), L / n


def vacuum_free(left, right, gamma=GAMMA):
    """True when the exact 1-D Riemann problem between two (rho, u, p) states
    creates no vacuum: 2/(gamma-1)(a_L + a_R) > u_R - u_L."""
    aL = np.sqrt(gamma * left[2] / left[0])
    aR = np.sqrt(gamma * right[2] / right[0])
    return 2.0 / (gamma - 1.0) * (aL + aR) > right[1] - left[1]


def riemann_instances(n_inst=256, dim=1, seed=1, size_range=None, gamma=GAMMA,
                      rho_range=(0.1, 10.0), p_range=(0.01, 1000.0), vel_range=(-2.0, 2.0)):
    """Seeded set of uneven-size Riemann instances for batched runs.

    1-D: size N ~ U{64..1024}, two states split at x = 1/2.
    2-D: size N ~ U{64..512}, N x N, four quadrant states split at (1/2, 1/2).
    rho, p log-uniform, velocities uniform.  A draw whose states would create
    vacuum in the exact 1-D Riemann problem between any two adjacent states is
    rejected and redrawn; the number of rejections is returned.
    Returns (list of (W, dx)), rejections, list of states.
    """
    rng = np.random.default_rng(seed)
    if size_range is None:
        size_range = (64, 1024) if dim == 1 else (64, 512)
    out, states, rej = [], [], 0

    def draw():
        rho = float(np.exp(rng.uniform(np.log(rho_range[0]), np.log(rho_range[1]))))
        vel = [float(rng.uniform(*vel_range)) for _ in range(dim)]
        p = float(np.exp(rng.uniform(np.log(p_range[0]), np.log(p_range[1]))))
        return rho, vel, p

    for _ in range(n_inst):
        n = int(rng.integers(size_range[0], size_range[1] + 1))
        while True:
            if dim == 1:
                sL, sR = draw(), draw()
                ok = vacuum_free((sL[0], sL[1][0], sL[2]), (sR[0], sR[1][0], sR[2]), gamma)
                st = (sL, sR)
            else:
                q = [draw() for _ in range(4)]
                # adjacent pairs across x = 1/2 (normal velocity u) and y = 1/2 (normal velocity v)
                pairs = [(q[0], q[1], 0), (q[3], q[2], 0), (q[0], q[3], 1), (q[1], q[2], 1)]
                ok = all(vacuum_free((a[0], a[1][k], a[2]), (b[0], b[1][k], b[2]), gamma)
                         for a, b, k in pairs)
                st = tuple(q)
            if ok:
                break
            rej += 1
        if dim == 1:
            W, dx = riemann_1d(n, (st[0][0], st[0][1][0], st[0][2]), (st[1][0], st[1][1][0], st[1][2]), gamma=gamma)
        else:
            W = quadrant_field(n, n, [(s[0], s[1][0], s[1][1], s[2]) for s in st], gamma=gamma)
            dx = 1.0 / n
        out.append((W, dx))
        states.append(st)
    return out, rej, states
