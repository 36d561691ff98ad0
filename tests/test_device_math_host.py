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
