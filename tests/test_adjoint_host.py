"""Reverse of the Gauss-point flux, checked on the host (no GPU).

The library's hand-written reverse (the code its reverse kernels run,
evaluated on the host) must satisfy <Fb, J v> = <J^T Fb, v> with J v the
oracle's forward-mode derivative of its own, independently written flux
(dual numbers through the generic moment engine, dt constant)."""
import numpy as np
import pytest

from gpu_common import gpu_params, orc_params, problem


@pytest.fixture(scope="module")
def lib():
    import os

    from paper_2309_10534_amd import tgks
    if not os.path.exists(tgks.LIB_PATH):
        pytest.skip("libtgks.so not built")
    return tgks


def face_state(rng, D, gamma=1.4, jump=0.3):
    rho = 1.0 + jump * rng.uniform(-1, 1)
    p = 1.0 + jump * rng.uniform(-1, 1)
    u = 0.5 * rng.uniform(-1, 1, D)
    return np.concatenate([[rho], rho * u, [p / (gamma - 1) + 0.5 * rho * (u @ u)]])


CASES = [
    (1, "inviscid", 0.0, 1.0), (2, "inviscid", 0.0, 1.0), (3, "inviscid", 0.0, 1.0),
    (1, "zero", 0.0, 1.0), (2, "zero", 0.0, 1.0),
    (1, "viscous", 1e-3, 0.72), (2, "viscous", 1e-3, 0.72), (3, "viscous", 1e-3, 0.72),
    (2, "inviscid", 2e-3, 0.72),
]


@pytest.mark.parametrize("D,tau,mu,pr", CASES)
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_flux_vjp_matches_oracle_jvp(orc, lib, D, tau, mu, pr, seed):
    rng = np.random.default_rng(100 * D + seed)
    nc = D + 2
    pr_ = problem([8] * D, [0.1] * D, tau=tau, mu=mu, prandtl=pr)
    Pg, Po = gpu_params(pr_), orc_params(orc, pr_)
    Wl, Wr = face_state(rng, D), face_state(rng, D)
    dWl = 0.5 * rng.uniform(-1, 1, (D, nc))
    dWr = 0.5 * rng.uniform(-1, 1, (D, nc))
    dt = 0.01
    Fb = rng.uniform(-1, 1, (2, nc))
    t = [rng.uniform(-1, 1, nc), rng.uniform(-1, 1, nc), rng.uniform(-1, 1, (D, nc)), rng.uniform(-1, 1, (D, nc))]
    F, dF = orc.gp_flux_dual(Po, Wl, Wr, dWl, dWr, *t, dt, [dt, 0.5 * dt])
    lhs = float(np.sum(Fb * dF))
    g = lib.tgks_gp_flux_vjp_host(Pg, Wl, Wr, dWl, dWr, dt, Fb)
    rhs = float(sum(np.sum(a * b) for a, b in zip(g, t)))
    scale = float(np.sum(np.abs(Fb * dF)))
    assert abs(lhs - rhs) <= 1e-11 * scale, (lhs, rhs)


def test_flux_vjp_finite_differences(lib):
    """Independent of the oracle: central differences of the library's own
    forward flux along random directions (2-D, inviscid)."""
    rng = np.random.default_rng(7)
    D, nc = 2, 4
    P = gpu_params(problem([8, 8], [0.1, 0.1]))
    Wl, Wr = face_state(rng, D), face_state(rng, D)
    dWl, dWr = 0.5 * rng.uniform(-1, 1, (D, nc)), 0.5 * rng.uniform(-1, 1, (D, nc))
    dt = 0.01
    Fb = rng.uniform(-1, 1, (2, nc))
    g = lib.tgks_gp_flux_vjp_host(P, Wl, Wr, dWl, dWr, dt, Fb)
    for _ in range(4):
        t = [rng.uniform(-1, 1, nc), rng.uniform(-1, 1, nc), rng.uniform(-1, 1, (D, nc)), rng.uniform(-1, 1, (D, nc))]
        h = 1e-6

        def f(s):
            F, ok = lib.tgks_gp_flux_host(P, Wl + s * t[0], Wr + s * t[1], dWl + s * t[2], dWr + s * t[3], dt)
            assert ok
            return F

        fd = (f(h) - f(-h)) / (2 * h)
        lhs = float(np.sum(Fb * fd))
        rhs = float(sum(np.sum(a * b) for a, b in zip(g, t)))
        assert abs(lhs - rhs) <= 1e-7 * max(abs(lhs), 1e-3)
