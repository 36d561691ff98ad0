"""Pins of the oracle's gas-kinetic flux (Sec. 2.1, Eqs. 2.2-2.9; kinetic
weighting Eqs. 3.25-3.26; collision time Sec. 5) against numerical quadrature
and closed-form special cases that do not use any of the oracle's formulas."""
import math

import numpy as np
import pytest
from scipy import integrate

from kinetic_quadrature import Gauss, gp_flux_quadrature, moment_matrix, psi_list
from paper_2309_10534_amd.inputs import conservative

GAMMA = 1.4


def rand_state(rng, D):
    rho = rng.uniform(0.3, 3.0)
    vel = [np.array([rng.uniform(-1.5, 1.5)]) for _ in range(D)]
    p = rng.uniform(0.2, 3.0)
    return conservative(np.array([rho]), vel, np.array([p]))[:, 0]


@pytest.mark.parametrize("kind", [0, 1, -1])
def test_maxwellian_moments_quadrature(orc, kind):
    rng = np.random.default_rng(20 + kind)
    for _ in range(10):
        U, lam = rng.uniform(-3, 3), rng.uniform(0.05, 5.0)
        m = orc.moments(U, lam, kind)
        lo, hi = {0: (-np.inf, np.inf), 1: (0.0, np.inf), -1: (-np.inf, 0.0)}[kind]
        for n in range(8):
            want = integrate.quad(lambda u: u ** n * math.sqrt(lam / math.pi) * math.exp(-lam * (u - U) ** 2),
                                  lo, hi, epsabs=1e-300, epsrel=1e-13, limit=200)[0]
            scale = integrate.quad(lambda u: abs(u) ** n * math.sqrt(lam / math.pi) * math.exp(-lam * (u - U) ** 2),
                                   -np.inf, np.inf, epsrel=1e-12)[0]
            assert abs(m[n] - want) <= 1e-13 * scale + 1e-300, (n, m[n], want)


def test_half_moments_sum_to_full(orc):
    rng = np.random.default_rng(2)
    for _ in range(20):
        U, lam = rng.uniform(-3, 3), rng.uniform(0.05, 5.0)
        np.testing.assert_allclose(orc.moments(U, lam, 1) + orc.moments(U, lam, -1), orc.moments(U, lam, 0),
                                   rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("D", [1, 2, 3])
def test_micro_slope_solve_residual(orc, D):
    rng = np.random.default_rng(30 + D)
    psis = psi_list(D)
    for _ in range(5):
        W = rand_state(rng, D)
        b = rng.normal(size=D + 2)
        a = orc.micro_slope(D, GAMMA, W, b)
        M = moment_matrix(Gauss(W, D, GAMMA), psis)
        np.testing.assert_allclose(M @ a, b, rtol=1e-11, atol=1e-11 * np.abs(b).max())


CASES = [(D, mode) for D in (1, 2, 3) for mode in ("inviscid", "viscous", "zero")]


@pytest.mark.parametrize("D,mode", CASES)
def test_gauss_point_flux_against_quadrature(orc, D, mode):
    """Whole Gauss-point flux: W0, dW0 (Eq. 2.6), micro slopes (Eq. 2.7), the
    time-integrated flux of Eq. 2.5 over dt and dt/2 and, for Navier-Stokes,
    the Prandtl correction of the energy flux."""
    rng = np.random.default_rng(100 + 3 * D + len(mode))
    mu, pr = (0.05, 0.72) if mode == "viscous" else (0.0, 1.0)
    for _ in range(2):
        Wl, Wr = rand_state(rng, D), rand_state(rng, D)
        dWl = rng.normal(size=(D, D + 2)) * 0.4
        dWr = rng.normal(size=(D, D + 2)) * 0.4
        dt = rng.uniform(0.002, 0.05)
        P = orc.make_params([8] * D, [0.1] * D, tau=mode, mu=mu, prandtl=pr)
        F, W0, dW0, bad = orc.gp_flux(P, Wl, Wr, dWl, dWr, dt, [dt, dt / 2])
        Fq, W0q, dW0q, tau = gp_flux_quadrature(D, GAMMA, Wl, Wr, dWl, dWr, dt, [dt, dt / 2],
                                                tau_mode=mode, mu=mu, prandtl=pr)
        assert bad == 0
        np.testing.assert_allclose(W0, W0q, rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(dW0, dW0q, rtol=1e-10, atol=1e-11 * np.abs(dW0q).max())
        np.testing.assert_allclose(F, Fq, rtol=1e-10, atol=1e-11 * np.abs(Fq).max())


@pytest.mark.parametrize("D", [1, 2, 3])
def test_kinetic_weighting_identity(orc, D):
    # equal left/right states and slopes: W0 = W and dW0 = dW (Eq. 2.6)
    rng = np.random.default_rng(40 + D)
    W = rand_state(rng, D)
    dW = rng.normal(size=(D, D + 2))
    P = orc.make_params([8] * D, [0.1] * D)
    F, W0, dW0, bad = orc.gp_flux(P, W, W, dW, dW, 0.01, [0.01])
    np.testing.assert_allclose(W0, W, rtol=1e-13)
    np.testing.assert_allclose(dW0, dW, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("D", [1, 2, 3])
@pytest.mark.parametrize("mode", ["inviscid", "zero", "viscous"])
def test_uniform_state_euler_flux(orc, D, mode):
    # uniform state: F(delta) = delta * Euler flux (C1 + C4 = delta)
    rng = np.random.default_rng(50 + D)
    W = rand_state(rng, D)
    rho, u = W[0], W[1:1 + D] / W[0]
    p = (GAMMA - 1) * (W[D + 1] - 0.5 * rho * np.dot(u, u))
    euler = np.concatenate([[rho * u[0]], rho * u[0] * u + p * np.eye(D)[0], [u[0] * (W[D + 1] + p)]])
    P = orc.make_params([8] * D, [0.1] * D, tau=mode, mu=0.01 if mode == "viscous" else 0.0,
                        prandtl=0.72 if mode == "viscous" else 1.0)
    z = np.zeros((D, D + 2))
    for delta in (0.01, 0.003):
        F, W0, dW0, bad = orc.gp_flux(P, W, W, z, z, 0.01, [delta])
        np.testing.assert_allclose(F[0], delta * euler, rtol=1e-13, atol=1e-15)


def test_failure_count(orc):
    P = orc.make_params([8], [0.1])
    good = conservative(np.array([1.0]), [np.array([0.0])], np.array([1.0]))[:, 0]
    badW = good.copy()
    badW[2] = 0.1 * badW[2] - 1.0  # negative internal energy
    z = np.zeros((1, 3))
    assert orc.gp_flux(P, good, good, z, z, 0.01, [0.01])[3] == 0
    assert orc.gp_flux(P, good, badW, z, z, 0.01, [0.01])[3] == 1
