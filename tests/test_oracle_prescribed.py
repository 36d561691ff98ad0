"""Pins of the prescribed (Dirichlet) sides of the double Mach reflection
(Sec. 5.7): inflow behind a shock keeps the totals on the grid on the
Rankine-Hugoniot law (exactly while the inflow cells stay uniform), an
oblique shock translates at its exact speed when every side follows its
motion (and lags at the top when the top's time dependence is dropped), and
a side whose line never admits state A reduces to its far kind exactly."""
import math

import numpy as np

from paper_2309_10534_amd import inputs as I

GAMMA = 1.4


def shock_states(ms, rho1=1.4, p1=1.0, gamma=GAMMA):
    """Post-shock (rho, u, p) behind a shock of Mach ms moving right into
    (rho1, 0, p1), and its speed (normal-shock relations)."""
    c1 = math.sqrt(gamma * p1 / rho1)
    m2 = ms * ms
    rho2 = rho1 * (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    p2 = p1 * (2.0 * gamma * m2 - (gamma - 1.0)) / (gamma + 1.0)
    S = ms * c1
    u2 = S * (1.0 - rho1 / rho2)
    return (rho2, u2, p2), S


def test_normal_shock_relations():
    """The Mach 10 post-shock state of the double Mach reflection."""
    (rho2, u2, p2), S = shock_states(10.0)
    assert abs(rho2 - 8.0) < 1e-12 and abs(p2 - 116.5) < 1e-12 and abs(S - 10.0) < 1e-12
    assert abs(u2 - 8.25) < 1e-12
    assert abs(math.hypot(*I.DMR_POST[1:3]) - 8.25) < 1e-12


def test_inflow_shock_1d(orc):
    """The post-shock state of a Mach 3 shock prescribed at the left end.
    (a) Shock started inside the grid, on a face: the post-shock flow is
    supersonic, so the cells at the inflow stay uniform, the inflow face
    carries exactly the flux of the prescribed state, and the mass,
    momentum and energy on the grid follow the Rankine-Hugoniot law to
    rounding.  (b) Gas at rest everywhere: the inflow forms the shock at the
    boundary; the totals then follow the law within a tenth of a cell (the
    start-up of the shock at the boundary face), while a transmissive end
    keeps the gas at rest."""
    (rho2, u2, p2), S = shock_states(3.0)
    assert u2 > math.sqrt(GAMMA * p2 / rho2)  # supersonic post-shock flow
    n, L = 200, 1.0
    dx = L / n
    B = I.conservative(np.full(n, 1.4), [np.zeros(n)], np.full(n, 1.0))
    A = I.conservative(np.array(rho2), [np.array(u2)], np.array(p2))
    P = orc.make_params([n], [dx], bc=[("prescribed", "transmissive")], states=(A.tolist(), [0, 0, 0]),
                        lines={(0, 0): (np.inf, 0.0, 0.0)})
    x0 = 0.2
    W0 = B.copy()
    W0[:, : int(round(x0 / dx))] = A[:, None]
    W, t, s, bad = orc.run(P, W0, 100000, cfl=0.5, t_end=0.04)
    assert bad == 0 and abs(t - 0.04) < 1e-14
    for c in range(3):
        exact = B[c][0] * L + (A[c] - B[c][0]) * (x0 + S * t)
        assert abs(W[c].sum() * dx - exact) < 1e-13 * abs(exact), c
    W, t, s, bad = orc.run(P, B, 100000, cfl=0.5, t_end=0.04)
    assert bad == 0
    for c in range(3):
        exact = B[c][0] * L + (A[c] - B[c][0]) * S * t
        assert abs(W[c].sum() * dx - exact) < 0.1 * abs(A[c] - B[c][0]) * dx, c
    x = (np.arange(n) + 0.5) * dx
    mid = (x > 0.25 * S * t) & (x < 0.75 * S * t)
    assert np.abs(W[0][mid] / rho2 - 1.0).max() < 0.05
    Pt = orc.make_params([n], [dx], bc="transmissive")
    W2, _, _, _ = orc.run(Pt, B, 100000, cfl=0.5, t_end=0.04)
    assert np.abs(W2 - B).max() < 1e-13


def oblique_shock_params(orc, nx, ny, ms, top_moves=True):
    """A Mach ms shock at 60 degrees to the x axis into (1.4, 0, 0, 1), every
    side following its exact motion x = 1/6 + (y + 2 S t) / sqrt 3."""
    (rho2, un, p2), S = shock_states(ms)
    post = (rho2, un * math.sqrt(3.0) / 2.0, -0.5 * un, p2)  # along the shock normal
    W, (dx, dy), A, B = I.oblique_shock(nx, ny, post, I.DMR_PRE)
    s3 = math.sqrt(3.0)
    line = (1.0 / 6.0, 1.0 / s3, 2.0 * S / s3)
    top = line if top_moves else (1.0 / 6.0, 1.0 / s3, 0.0)
    P = orc.make_params([nx, ny], [dx, dy], bc=[("prescribed", "transmissive"), ("prescribed", "prescribed")],
                        states=(A.tolist(), B.tolist()),
                        lines={(0, 0): (np.inf, 0.0, 0.0), (1, 0): line, (1, 1): top},
                        far={(1, 0): "state_b", (1, 1): "state_b"})
    return P, W, dx, dy, S, rho2


def row_shock_positions(W, dx, rho_a, rho_b=1.4):
    Lx = W.shape[2] * dx
    return (W[0].sum(axis=1) * dx - rho_b * Lx) / (rho_a - rho_b)


def test_oblique_shock_translates(orc):
    """Every side follows the exact moving Mach 1.5 shock (no wall): the
    solution is the oblique shock moving at 2 S / sqrt 3 along x, and the
    mass-equivalent shock position of every row stays within a quarter cell of the
    exact line.  With the top's states frozen at t = 0 the rows next to the
    top fall behind."""
    nx, ny, t_end = 96, 24, 0.25
    P, W0, dx, dy, S, rho2 = oblique_shock_params(orc, nx, ny, 1.5)
    W, t, s, bad = orc.run(P, W0, 100000, cfl=0.5, t_end=t_end)
    assert bad == 0 and abs(t - t_end) < 1e-14
    y = (np.arange(ny) + 0.5) * dy
    exact = 1.0 / 6.0 + (y + 2.0 * S * t) / math.sqrt(3.0)
    assert exact.min() > 10 * dx and exact.max() < 4.0 - 10 * dx
    err = np.abs(row_shock_positions(W, dx, rho2) - exact)
    assert err.max() < 0.25 * dx, err / dx
    P2, _, _, _, _, _ = oblique_shock_params(orc, nx, ny, 1.5, top_moves=False)
    W2, _, _, bad2 = orc.run(P2, W0, 100000, cfl=0.5, t_end=t_end)
    err2 = np.abs(row_shock_positions(W2, dx, rho2) - exact)
    assert err2[-1] > 5.0 * dx and err2[: ny // 2].max() < 0.25 * dx, err2 / dx


def test_far_kinds_reduce_to_plain_sides(orc):
    """A prescribed side whose line never admits state A (s0 = -inf) is its
    far kind: reflective and transmissive far kinds give bit-identical
    steps to the plain sides; far state B equals a prescribed side whose
    line always admits A = B."""
    rng = np.random.default_rng(5)
    nx, ny = 20, 12
    rho = 1.0 + 0.3 * rng.random((ny, nx))
    W = I.conservative(rho, [0.5 * rng.standard_normal((ny, nx)), 0.5 * rng.standard_normal((ny, nx))],
                       1.0 + 0.3 * rng.random((ny, nx)))
    dxs = [1.0 / nx, 1.0 / ny]
    never = (-np.inf, 0.0, 0.0)
    for far in ("reflective", "transmissive"):
        Pp = orc.make_params([nx, ny], dxs, bc=[("prescribed", "prescribed"), ("prescribed", "prescribed")],
                             lines={(d, e): never for d in range(2) for e in range(2)},
                             far={(d, e): far for d in range(2) for e in range(2)})
        Pr = orc.make_params([nx, ny], dxs, bc=far)
        dt = orc.cfl_dt(Pr, W, 0.5)
        a, fa, _, _ = orc.step(Pp, W, dt, want_flags=True, t=0.37)
        b, fb, _, _ = orc.step(Pr, W, dt, want_flags=True)
        assert np.array_equal(a, b) and np.array_equal(fa, fb), far
    S = [1.1, 0.2, -0.3, 2.5]
    P1 = orc.make_params([nx, ny], dxs, bc="prescribed", states=([0, 0, 0, 0], S),
                         lines={(d, e): never for d in range(2) for e in range(2)})
    P2 = orc.make_params([nx, ny], dxs, bc="prescribed", states=(S, [0, 0, 0, 0]),
                         lines={(d, e): (np.inf, 0.0, 0.0) for d in range(2) for e in range(2)})
    dt = orc.cfl_dt(P1, W, 0.5)
    assert np.array_equal(orc.step(P1, W, dt)[0], orc.step(P2, W, dt)[0])
    # and the prescribed state does reach the interior
    Pt = orc.make_params([nx, ny], dxs, bc="transmissive")
    assert not np.array_equal(orc.step(P1, W, dt)[0], orc.step(Pt, W, dt)[0])


def test_three_dimensions_rejected(orc):
    import pytest
    P = orc.make_params([6, 6, 6], [0.1] * 3, bc="prescribed")
    with pytest.raises(ValueError):
        orc.step(P, np.ones((5, 6, 6, 6)), 1e-3)
