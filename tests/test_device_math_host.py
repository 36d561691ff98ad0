"""The device Gauss-point flux (closed-form moments, Jacobian-vector
products of the Euler flux and of the second-moment flux, closed-form
micro-slope solves), evaluated on the host through tgks_gp_flux_host, against
the oracle's generic moment engine.  No device needed."""
import os

import numpy as np
import pytest

from paper_2309_10534_amd.inputs import conservative


@pytest.fixture(scope="module")
def tg():
    from paper_2309_10534_amd import tgks
    if not os.path.exists(tgks.LIB_PATH):
        pytest.skip("libtgks.so not built")
    return tgks


def rand_state(rng, D):
    return conservative(np.array([rng.uniform(0.3, 3.0)]), [np.array([rng.uniform(-1.5, 1.5)]) for _ in range(D)],
                        np.array([rng.uniform(0.2, 3.0)]))[:, 0]


@pytest.mark.parametrize("D", [1, 2, 3])
@pytest.mark.parametrize("mode", ["inviscid", "viscous", "zero"])
def test_device_flux_matches_oracle(orc, tg, D, mode):
    rng = np.random.default_rng(7 + D + len(mode))
    mu, pr = (0.05, 0.72) if mode == "viscous" else (0.0, 1.0)
    P = orc.make_params([8] * D, [0.1] * D, tau=mode, mu=mu, prandtl=pr)
    Pg = tg.tgks_params_default(D, [8] * D, [0.1] * D, tau=mode, mu=mu, prandtl=pr)
    for _ in range(20):
        Wl, Wr = rand_state(rng, D), rand_state(rng, D)
        dWl = rng.normal(size=(D, D + 2)) * 0.5
        dWr = rng.normal(size=(D, D + 2)) * 0.5
        dt = rng.uniform(1e-3, 0.05)
        Fo, _, _, bad = orc.gp_flux(P, Wl, Wr, dWl, dWr, dt, [dt, dt / 2])
        Fg, ok = tg.tgks_gp_flux_host(Pg, Wl, Wr, dWl, dWr, dt)
        assert ok and bad == 0
        np.testing.assert_allclose(Fg, Fo, rtol=1e-12, atol=1e-13 * np.abs(Fo).max())


def test_device_flux_flags_nonphysical(tg):
    Pg = tg.tgks_params_default(1, [8], [0.1])
    good = conservative(np.array([1.0]), [np.array([0.2])], np.array([1.0]))[:, 0]
    bad = good.copy()
    bad[2] = -1.0
    assert tg.tgks_gp_flux_host(Pg, good, good, np.zeros(3), np.zeros(3), 0.01)[1]
    assert not tg.tgks_gp_flux_host(Pg, good, bad, np.zeros(3), np.zeros(3), 0.01)[1]


def stencils(rng, n):
    """Five-value stencils of every kind the selection meets: smooth, jumps,
    constants (exact and with last-bit noise), linear ramps, huge and tiny
    magnitudes, NaN and infinity."""
    out = []
    for i in range(n):
        k = i % 9
        if k == 0:
            Q = rng.normal(size=5)
        elif k == 1:
            Q = 1.0 + 0.01 * np.sin(rng.uniform(0, 6) + 0.2 * np.arange(5))
        elif k == 2:
            Q = np.where(np.arange(5) < rng.integers(1, 5), 1.0, 0.1) + 1e-4 * rng.normal(size=5)
        elif k == 3:
            Q = np.full(5, rng.choice([0.7, 1.0, 3.3]))
        elif k == 4:
            Q = np.full(5, 0.7) * (1 + rng.choice([0.0, 1.1e-16, -2.2e-16], size=5))
        elif k == 5:
            Q = rng.uniform(-1, 1) + rng.uniform(-1, 1) * np.arange(5.0)
        elif k == 6:
            Q = rng.normal(size=5) * 10.0 ** rng.uniform(-30, 30)
        elif k == 7:
            Q = 1.0 + rng.normal(size=5) * 10.0 ** rng.integers(-8, -2)
        else:
            Q = rng.normal(size=5)
            Q[rng.integers(0, 5)] = rng.choice([np.nan, np.inf, -np.inf, 1e200])
        out.append(Q)
    return out


@pytest.mark.parametrize("ct1", [1e-7, 1e-5, 0.25])
def test_teno_flag_shortcut_is_exact(orc, ct1):
    """The kernels decide certain large-stencil selections without the
    weights (b_3 <= 4 b_k, C_T1 <= 1e-5); over stencils of every kind the
    flag equals the one from the weights of Eq. 4.5 bit for bit, and both
    equal the oracle's selection (finite inputs)."""
    from paper_2309_10534_amd import tgks
    p = tgks.tgks_params_default(1, [10], [0.1])
    p.ct1 = ct1
    rng = np.random.default_rng(7)
    n_fast = 0
    for Q in stencils(rng, 20000):
        a = tgks.tgks_teno_flag_host(p, Q, fast=True)
        b = tgks.tgks_teno_flag_host(p, Q, fast=False)
        assert a == b, Q
        if np.all(np.isfinite(Q)):
            assert a == orc.teno_select(Q, ct1=ct1), Q
        n_fast += a == 1
    assert n_fast > 2000
