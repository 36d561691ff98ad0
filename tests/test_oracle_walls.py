"""Pins of the no-slip adiabatic wall (the wall of the viscous shock tube,
Sec. 5.8): the impulsively started plate against its exact solution,
conservation of mass and energy in a closed box, rest preserved, and the
difference from the reflective (slip) wall."""
import math

import numpy as np
from scipy.special import erf

from paper_2309_10534_amd import inputs as I

GAMMA = 1.4


def rayleigh(orc, bottom, nu=2e-3, U=0.05, t_end=0.3, nx=3, ny=48, H=0.2):
    """Uniform flow U along a wall at y = 0 (periodic in x, symmetry at the
    top), constant viscosity; returns (y, u at t_end, t)."""
    dy = H / ny
    rho = np.ones((ny, nx))
    p = np.full((ny, nx), 1.0 / GAMMA)
    W = I.conservative(rho, [np.full((ny, nx), U), np.zeros((ny, nx))], p)
    P = orc.make_params([nx, ny], [dy, dy], bc=[("periodic", "periodic"), (bottom, "reflective")],
                        tau="viscous", mu=nu, prandtl=1.0)
    Wn, t, s, bad = orc.run(P, W, 100000, cfl=0.5, t_end=t_end)
    assert bad == 0 and abs(t - t_end) < 1e-12
    return (np.arange(ny) + 0.5) * dy, Wn[1][:, 0] / Wn[0][:, 0], t


def test_impulsively_started_plate(orc):
    """Stokes' first problem: at low Mach number the velocity beside a
    no-slip wall is U erf(y / (2 sqrt(nu t))); the reflective wall keeps the
    uniform flow."""
    U, nu = 0.05, 2e-3
    y, u, t = rayleigh(orc, "noslip", nu=nu, U=U)
    exact = U * erf(y / (2.0 * math.sqrt(nu * t)))
    assert np.abs(u - exact).max() < 5e-3 * U
    assert u[0] < 0.25 * U  # the wall drags the first cell
    y, u, t = rayleigh(orc, "reflective", nu=nu, U=U)
    assert np.abs(u - U).max() < 1e-12


def box_state(shape, seed):
    rng = np.random.default_rng(seed)
    sh = tuple(reversed(shape))
    grids = np.meshgrid(*[(np.arange(n) + 0.5) / n for n in reversed(shape)], indexing="ij")
    phase = sum((k + 1) * g for k, g in enumerate(grids))
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * phase) + 0.01 * rng.normal(size=sh)
    vel = [0.2 * np.cos(2 * np.pi * (phase + 0.3 * k)) for k in range(len(shape))]
    p = 1.0 + 0.1 * np.cos(2 * np.pi * phase)
    return I.conservative(rho, vel, p)


def test_closed_box_conserves_mass_and_energy(orc):
    """No mass or energy crosses an adiabatic no-slip wall: the two totals
    of a closed box are kept to rounding while the momentum is not."""
    for shape, steps in (([16, 12], 4), ([4, 4, 4], 1)):
        D = len(shape)
        W = box_state(shape, seed=D)
        dx = [1.0 / n for n in shape]
        P = orc.make_params(shape, dx, bc="noslip", tau="viscous", mu=5e-3, prandtl=0.72)
        W1 = W.copy()
        for _ in range(steps):
            W1, _, _, bad = orc.step(P, W1, orc.cfl_dt(P, W1, 0.5))
            assert bad == 0
        for c in (0, D + 1):
            assert abs(W1[c].sum() - W[c].sum()) <= 1e-13 * abs(W[c].sum()), (shape, c)
        assert abs(W1[1].sum() - W[1].sum()) > 1e-6 * np.abs(W[1]).sum()


def test_rest_is_preserved(orc):
    W = I.conservative(np.ones((10, 12)), [np.zeros((10, 12))] * 2, np.ones((10, 12)))
    P = orc.make_params([12, 10], [0.1, 0.1], bc="noslip", tau="viscous", mu=1e-2, prandtl=0.73)
    W1 = W.copy()
    for _ in range(3):
        W1, _, _, bad = orc.step(P, W1, orc.cfl_dt(P, W1, 0.5))
    assert bad == 0
    assert np.abs(W1[1:3]).max() < 1e-14 and np.abs(W1 - W).max() < 1e-13
