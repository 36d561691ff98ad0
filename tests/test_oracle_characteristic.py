"""Pins of the oracle's characteristic-variable reconstruction option.

The fields are the eigenvectors of the Euler flux Jacobian at the mean of
the two cells beside a face.  Pinned here against mathematics the option
does not share code with: the eigen-decomposition against a finite-
difference Jacobian of an independently written Euler flux, the exact
constancy of velocity and pressure across a contact (the acoustic fields of
a contact are constant), agreement with the conservative reconstruction
wherever every selection keeps the large (linear) stencil, and the exact
Sod solution."""
import math

import numpy as np
import pytest

from exact_riemann import cell_average_density
from paper_2309_10534_amd import inputs as I

GAMMA = 1.4


def euler_flux(W, a, gamma=GAMMA):
    """F_a(W) in frame order (rho, m_0..m_{D-1}, E), written out directly."""
    D = len(W) - 2
    rho, m, E = W[0], W[1:D + 1], W[D + 1]
    u = m / rho
    p = (gamma - 1.0) * (E - 0.5 * rho * (u @ u))
    F = np.empty_like(W)
    F[0] = m[a]
    F[1:D + 1] = m[a] * u
    F[1 + a] += p
    F[D + 1] = u[a] * (E + p)
    return F


def random_state(rng, D):
    rho = math.exp(rng.uniform(-1.0, 1.0))
    u = rng.uniform(-1.5, 1.5, D)
    p = math.exp(rng.uniform(-1.0, 1.0))
    return np.concatenate([[rho], rho * u, [p / (GAMMA - 1.0) + 0.5 * rho * (u @ u)]])


@pytest.mark.parametrize("D", [1, 2, 3])
def test_basis_inverse_and_diagonalises_jacobian(orc, D):
    rng = np.random.default_rng(10 + D)
    nc = D + 2
    for _ in range(20):
        Wb = random_state(rng, D)
        rho, u = Wb[0], Wb[1:D + 1] / Wb[0]
        p = (GAMMA - 1.0) * (Wb[-1] - 0.5 * rho * (u @ u))
        c = math.sqrt(GAMMA * p / rho)
        for a in range(D):
            L, R, ok = orc.char_basis(D, GAMMA, Wb, a)
            assert ok
            assert np.abs(L @ R - np.eye(nc)).max() < 1e-12
            # central differences of the flux, column by column
            J = np.empty((nc, nc))
            for j in range(nc):
                h = 1e-6 * max(1.0, abs(Wb[j]))
                e = np.zeros(nc)
                e[j] = h
                J[:, j] = (euler_flux(Wb + e, a) - euler_flux(Wb - e, a)) / (2 * h)
            lam = np.array([u[a] - c] + [u[a]] * D + [u[a] + c])
            A = R @ np.diag(lam) @ L
            assert np.abs(A - J).max() <= 1e-7 * max(1.0, np.abs(J).max()), (D, a)


def test_basis_nonphysical_is_identity(orc):
    Wb = np.array([1.0, 0.0, 0.0, -1.0])  # negative pressure
    L, R, ok = orc.char_basis(2, GAMMA, Wb, 0)
    assert not ok and np.array_equal(L, np.eye(4)) and np.array_equal(R, np.eye(4))


@pytest.mark.parametrize("D", [1, 2])
def test_contact_keeps_velocity_and_pressure(orc, D):
    """Across a contact (density jump, uniform velocity and pressure) the
    acoustic and shear fields are constant, so the characteristic
    reconstruction returns the uniform velocity and pressure on both sides
    of the face to rounding (a wrong eigenvector or field order mixes the
    jump into those fields)."""
    u = np.array([0.7, -0.3][:D])
    p = 0.9
    rho = np.array([1.0, 1.0, 1.0, 0.2, 0.2, 0.2])  # jump between cells f-1 and f
    cells = np.stack([np.concatenate([[r], r * u, [p / (GAMMA - 1.0) + 0.5 * r * (u @ u)]]) for r in rho])
    P = orc.make_params([16] * D, [0.1] * D, recon=1)
    out, _ = orc.char_recon(P, cells, 0.1)
    for s in (out[0], out[2]):
        vel = s[1:D + 1] / s[0]
        pr = (GAMMA - 1.0) * (s[-1] - 0.5 * (s[1:D + 1] @ s[1:D + 1]) / s[0])
        assert np.abs(vel - u).max() < 1e-13 and abs(pr - p) < 1e-13
    # the density keeps its two values on the two sides
    assert abs(out[0][0] - 1.0) < 1e-13 and abs(out[2][0] - 0.2) < 1e-13


def smooth_1d(n):
    x = (np.arange(n) + 0.5) / n
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * x)
    u = 0.5 + 0.1 * np.cos(2 * np.pi * x)
    p = 1.0 + 0.1 * np.sin(4 * np.pi * x)
    return I.conservative(rho, [u], p)


def smooth_2d(n):
    x = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(x, x)
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * (X + Y))
    u = 0.4 + 0.1 * np.cos(2 * np.pi * Y)
    v = -0.3 + 0.1 * np.sin(2 * np.pi * X)
    p = 1.0 + 0.1 * np.cos(2 * np.pi * (X - Y))
    return I.conservative(rho, [u, v], p)


def smooth_step(orc, D, n, recon):
    W = smooth_1d(n) if D == 1 else smooth_2d(n)
    P = orc.make_params([n] * D, [1.0 / n] * D, bc="periodic", recon=recon)
    dt = orc.cfl_dt(P, W, 0.5)
    Wn, fl, _, bad = orc.step(P, W, dt, want_flags=True)
    assert bad == 0
    return Wn, fl


def test_smooth_step_equals_conservative_1d(orc):
    """Where every selection keeps the large stencil the reconstruction is
    linear, the projection commutes with it, and one step in characteristic
    variables equals the step in conservative variables to rounding."""
    n = 48
    (W0, f0), (W1, f1) = smooth_step(orc, 1, n, 0), smooth_step(orc, 1, n, 1)
    assert np.all(f0 == 1) and np.all(f1 == 1)
    for c in range(3):
        assert np.abs(W1[c] - W0[c]).sum() <= 1e-14 * np.abs(W0[c]).sum()


def test_smooth_step_converges_to_conservative_2d(orc):
    """2-D: the normal selections all keep the large stencil, but along a
    face some fields (shear, normal slopes) are nearly constant and their
    selections are decided by rounding residues, so the two variants differ
    at truncation level; the difference falls at high order with the mesh."""
    diff = {}
    for n in (24, 48):
        (W0, f0), (W1, f1) = smooth_step(orc, 2, n, 0), smooth_step(orc, 2, n, 1)
        nn = 2 * 4 * n * n
        assert np.all(f0[:nn] == 1) and np.all(f1[:nn] == 1)
        diff[n] = max(np.abs(W1[c] - W0[c]).sum() / np.abs(W0[c]).sum() for c in range(4))
    assert diff[24] < 1e-7 and diff[48] < diff[24] / 16, diff


def test_sod_exact_riemann_characteristic(orc):
    """Sod with characteristic reconstruction converges to the exact solution
    like the conservative variant, with no overshoot."""
    errs = {}
    for n in (100, 400):
        W0, dx = I.sod(n)
        P = orc.make_params([n], [dx], recon=1)
        W, t, s, bad = orc.run(P, W0, 100000, cfl=0.5, t_end=0.2)
        assert bad == 0 and abs(t - 0.2) < 1e-13
        ex = cell_average_density((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), n, 0.2)
        errs[n] = np.mean(np.abs(W[0] - ex))
        rho, vel, p = I.primitive(W)
        assert rho.max() < 1.0 + 1e-3 and p.max() < 1.0 + 1e-3
        assert rho.min() > 0.1 and p.min() > 0.09
    assert errs[400] < 2.5e-3 and errs[100] > errs[400], errs


def test_three_dimensions_rejected(orc):
    P = orc.make_params([8, 8, 8], [0.1] * 3, recon=1)
    with pytest.raises(ValueError):
        orc.step(P, np.ones((5, 8, 8, 8)), 1e-3)
