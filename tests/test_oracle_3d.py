"""Pins of the oracle's 3-D assembly (Sec. 3.2 Steps 1-3 carried to three
dimensions as two tangential sweeps with 2 x 2 Gauss points, and the 3-D
kinetic constants of Sec. 2.1).

* Axis reduction.  A 3-D field that is uniform along one axis, with no
  velocity along it, is a 2-D flow: the Maxwellian's velocity along the
  uniform axis is one more Gaussian degree of freedom with the variance of
  the internal ones (K + D is the same), the faces normal to that axis carry
  identical fluxes, and the tangential sweep along it sees constant data.
  One 3-D step must therefore equal the oracle's 2-D step on the other two
  axes, for each of the three axes, with anisotropic cell widths: this pins
  both sweeps, the cyclic axis order, the Gauss-point weights and the
  per-axis slope scalings.
* Linear shear wave.  v = A sin(k z) (and its cyclic images) decays as
  exp(-nu k^2 t) under linearised Navier-Stokes.
"""
import math

import numpy as np
import pytest

from paper_2309_10534_amd import inputs as I

DX3 = (1 / 11, 1 / 13, 1 / 17)


def field_2d(nx, ny, dx, dy, seed):
    """Smooth 2-D flow with a mild slanted density jump (both selection
    branches of the sweeps are exercised)."""
    rng = np.random.default_rng(seed)
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    X, Y = np.meshgrid(x, y)
    a = rng.uniform(0.5, 1.5, size=6)
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * (a[0] * X + a[1] * Y)) + 0.3 * (X + 0.7 * Y > 0.45)
    u = 0.3 + 0.2 * np.cos(2 * np.pi * a[2] * Y)
    v = -0.2 + 0.15 * np.sin(2 * np.pi * a[3] * X)
    p = 1.0 + 0.1 * np.cos(2 * np.pi * (a[4] * X - a[5] * Y))
    return I.conservative(rho, [u, v], p)


def embed(W2, axis, n_uniform):
    """3-D state uniform along `axis` with zero momentum along it.  The two
    other axes (b, c), in cyclic order after `axis`, are the 2-D (x, y):
    axis 2 -> (x, y), axis 0 -> (y, z), axis 1 -> (z, x)."""
    b, c = (axis + 1) % 3, (axis + 2) % 3
    ny2, nx2 = W2.shape[1:]
    shape = [0, 0, 0]
    shape[b], shape[c], shape[axis] = nx2, ny2, n_uniform
    Z, Y, X = np.meshgrid(*[np.arange(shape[d]) for d in (2, 1, 0)], indexing="ij")
    pos = [X, Y, Z]
    W3 = np.zeros((5, shape[2], shape[1], shape[0]))
    for c3, c2 in ((0, 0), (1 + b, 1), (1 + c, 2), (4, 3)):
        W3[c3] = W2[c2][pos[c], pos[b]]
    return W3, shape


def reduce_slice(W3, axis, k):
    """Slice k along `axis` as a 2-D field (rho, m_b, m_c, E) on (b, c), and
    the momentum along `axis` there."""
    b, c = (axis + 1) % 3, (axis + 2) % 3
    nb, ncc = W3.shape[3 - b], W3.shape[3 - c]
    J, Ib = np.meshgrid(np.arange(ncc), np.arange(nb), indexing="ij")
    pos = [None, None, None]
    pos[axis], pos[b], pos[c] = np.full_like(J, k), Ib, J
    take = lambda F: F[pos[2], pos[1], pos[0]]
    return np.stack([take(W3[c3]) for c3 in (0, 1 + b, 1 + c, 4)]), take(W3[1 + axis])


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("ns", [False, True])
def test_axis_reduction_to_2d(orc, axis, ns):
    b, c = (axis + 1) % 3, (axis + 2) % 3
    nx2, ny2, nu = 10, 9, 4
    W2 = field_2d(nx2, ny2, DX3[b], DX3[c], seed=axis + 3 * ns)
    W3, shape = embed(W2, axis, nu)
    bc3 = [("periodic", "periodic")] * 3
    bc3[b] = ("transmissive", "reflective")
    bc3[c] = ("periodic", "periodic")
    kw = dict(tau="viscous", mu=2e-3, prandtl=0.72) if ns else {}
    P3 = orc.make_params(shape, DX3, bc=bc3, **kw)
    P2 = orc.make_params([nx2, ny2], [DX3[b], DX3[c]], bc=[bc3[b], bc3[c]], **kw)
    dt = 0.5 * orc.cfl_dt(P2, W2, 0.5)
    o3, _, s3, bad3 = orc.step(P3, W3, dt, want_wstar=True)
    o2, _, s2, bad2 = orc.step(P2, W2, dt, want_wstar=True)
    assert bad3 == bad2 == 0
    scale = np.abs(W2).reshape(4, -1).max(axis=1)[:, None, None]
    for k in range(nu):
        for got3, want2 in ((o3, o2), (s3, s2)):
            r, ma = reduce_slice(got3, axis, k)
            err = np.abs(r - want2) / scale
            assert err.max() <= 1e-13, (axis, k, err.max())
            assert np.abs(ma).max() <= 1e-14
    # the slices along the uniform axis are identical to rounding
    r0, _ = reduce_slice(o3, axis, 0)
    r1, _ = reduce_slice(o3, axis, nu - 1)
    assert np.abs(r0 - r1).max() <= 1e-14 * scale.max()


def test_axis_reduction_detects_spacing_swap(orc):
    """The reduction is sensitive to the per-axis scalings: the same 3-D
    field stepped with the uniform axis's width changed is unchanged, while
    swapping the widths of the two active axes changes the result."""
    axis = 2
    W2 = field_2d(10, 9, DX3[0], DX3[1], seed=11)
    W3, shape = embed(W2, axis, 4)
    P3 = orc.make_params(shape, DX3, bc="periodic")
    dt = 1e-3
    a, _, _, _ = orc.step(P3, W3, dt)
    P3b = orc.make_params(shape, (DX3[0], DX3[1], 0.3), bc="periodic")
    b, _, _, _ = orc.step(P3b, W3, dt)
    assert np.abs(a - b).max() <= 1e-14
    P3c = orc.make_params(shape, (DX3[1], DX3[0], DX3[2]), bc="periodic")
    c, _, _, _ = orc.step(P3c, W3, dt)
    assert np.abs(a - c).max() > 1e-6


def cell_avg_sin(n, k):
    x = (np.arange(n) + 0.5) / n
    return x, (np.cos(k * (x - 0.5 / n)) - np.cos(k * (x + 0.5 / n))) / (k / n)


@pytest.mark.parametrize("var_axis", [0, 1, 2])
def test_ns_shear_wave_decay_3d(orc, var_axis):
    """Linearised Navier-Stokes in 3-D: the velocity along the axis after
    var_axis (cyclic), A sin(k x_var), decays as exp(-nu k^2 t)."""
    n, mu, A = 24, 0.01, 1e-3
    k = 2 * np.pi
    x, s = cell_avg_sin(n, k)
    shape = [3, 3, 3]
    shape[var_axis] = n
    vel_axis = (var_axis + 1) % 3
    bshape = [1, 1, 1]
    bshape[2 - var_axis] = n
    prof = np.broadcast_to((A * s).reshape(bshape), (shape[2], shape[1], shape[0]))
    vel = [np.zeros_like(prof) for _ in range(3)]
    vel[vel_axis] = prof
    one = np.ones_like(prof)
    W = I.conservative(one, vel, one)
    dx = [1 / 3, 1 / 3, 1 / 3]
    dx[var_axis] = 1 / n
    P = orc.make_params(shape, dx, bc="periodic", tau="viscous", mu=mu, prandtl=0.72)
    T = 0.1
    Wn, t, steps, bad = orc.run(P, W, 10000, cfl=0.5, t_end=T)
    assert bad == 0 and abs(t - T) < 1e-13
    sl = [1, 1, 1]
    sl[2 - var_axis] = slice(None)
    got = Wn[1 + vel_axis][tuple(sl)]
    ratio = 2 * np.mean(got * np.sin(k * x)) / (2 * np.mean(prof[tuple(sl)] * np.sin(k * x)))
    assert abs(ratio / math.exp(-mu * k * k * T) - 1) < 3e-3, (var_axis, ratio)
    # the other velocity components are driven only at second order in A
    # (viscous heating of the shear layer)
    for a in range(3):
        if a != vel_axis:
            assert np.abs(Wn[1 + a]).max() < 1e-3 * A


def trilinear(coef, x, y, z):
    """sum over (i, j, k) in {0, 1}^3 of coef[k, j, i] x^i y^j z^k, and its
    gradient (d/dx, d/dy, d/dz)."""
    v = sum(coef[k, j, i] * x ** i * y ** j * z ** k for i in (0, 1) for j in (0, 1) for k in (0, 1))
    g = [sum(coef[k, j, 1] * y ** j * z ** k for j in (0, 1) for k in (0, 1)),
         sum(coef[k, 1, i] * x ** i * z ** k for i in (0, 1) for k in (0, 1)),
         sum(coef[1, j, i] * x ** i * y ** j for i in (0, 1) for j in (0, 1))]
    return v, g


@pytest.mark.parametrize("ns", [False, True])
def test_trilinear_field_exact_assembly(orc, ns):
    """Brute force on a trilinear field.  Every one-dimensional
    reconstruction the 3-D assembly makes (along the normal, then the two
    tangential sweeps) sees data that are linear along its axis, which every
    candidate polynomial reproduces exactly, and cell and face averages of a
    trilinear function are its centre values.  The Gauss-point states and
    their three derivatives are therefore the field's own values and
    gradients at (x_f, y_g, z_g), whatever the stencil selection.  Stage 1
    of the step (W*) of every cell whose stencils stay inside the grid must
    equal W - sum_d (F_d+ - F_d-) / dx_d with each face flux the mean of the
    Gauss-point fluxes of these exact states at the four points
    (+-1/(2 sqrt 3) of the face's two widths): a Gauss-point, sweep or
    spacing mix-up that needs both tangential axes to show fails here."""
    rng = np.random.default_rng(21)
    n = (9, 10, 11)
    dx = DX3
    # trilinear rho, rho U, rho V, rho W, rho E with small gradients about a
    # physical state
    base = np.array([1.0, 0.3, -0.2, 0.25, 2.6])
    coefs = []
    for c in range(5):
        co = rng.uniform(-0.15, 0.15, size=(2, 2, 2)) * (1.0 if c != 4 else 2.0)
        co[0, 0, 0] = base[c]
        coefs.append(co)
    Z, Y, X = np.meshgrid(*[(np.arange(n[d]) + 0.5) * dx[d] for d in (2, 1, 0)], indexing="ij")
    W = np.stack([trilinear(coefs[c], X, Y, Z)[0] for c in range(5)])
    kw = dict(tau="viscous", mu=2e-3, prandtl=0.72) if ns else {}
    P = orc.make_params(list(n), list(dx), bc="transmissive", **kw)
    dt = 2e-3
    _, _, Ws, bad = orc.step(P, W, dt, want_wstar=True)
    assert bad == 0
    g = 0.5 / math.sqrt(3.0)

    def face_flux(d, pos):
        t1, t2 = (d + 1) % 3, (d + 2) % 3
        perm = [0, 1 + d, 1 + t1, 1 + t2, 4]
        axes = [d, t1, t2]
        F = np.zeros(5)
        for s1 in (-1, 1):
            for s2 in (-1, 1):
                pt = list(pos)
                pt[t1] += s1 * g * dx[t1]
                pt[t2] += s2 * g * dx[t2]
                vals = [trilinear(coefs[c], *pt) for c in range(5)]
                Wf = np.array([vals[perm[a]][0] for a in range(5)])
                dWf = np.array([[vals[perm[a]][1][axes[e]] for a in range(5)] for e in range(3)])
                Fg, _, _, b = orc.gp_flux(P, Wf, Wf, dWf, dWf, dt, [0.5 * dt])
                assert b == 0
                F[perm] += 0.25 * Fg[0]
        return F

    scale = np.abs(W).reshape(5, -1).max(axis=1)
    worst = 0.0
    for k in range(3, n[2] - 3):
        for j in range(3, n[1] - 3):
            for i in range(3, n[0] - 3):
                ctr = [(i + 0.5) * dx[0], (j + 0.5) * dx[1], (k + 0.5) * dx[2]]
                want = W[:, k, j, i].copy()
                for d in range(3):
                    lo, hi = list(ctr), list(ctr)
                    lo[d] -= 0.5 * dx[d]
                    hi[d] += 0.5 * dx[d]
                    want -= (face_flux(d, hi) - face_flux(d, lo)) / dx[d]
                err = np.abs(Ws[:, k, j, i] - want) / scale
                worst = max(worst, err.max())
    assert worst <= 1e-12, worst
