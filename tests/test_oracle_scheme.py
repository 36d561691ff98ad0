"""Whole-scheme pins of the oracle: exact Sod solution, conservation,
symmetries, free-stream preservation, Navier-Stokes decay rates, forward-mode
derivatives against finite differences, boundary handling and failure
counting."""
import math

import numpy as np
import pytest

from exact_riemann import cell_average_density
from paper_2309_10534_amd import inputs as I

GAMMA = 1.4


def sod_l1(orc, n):
    W0, dx = I.sod(n)
    P = orc.make_params([n], [dx], bc="transmissive")
    W, t, s, bad = orc.run(P, W0, 100000, cfl=0.5, t_end=0.2)
    assert bad == 0 and abs(t - 0.2) < 1e-13
    ex = cell_average_density((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), n, 0.2)
    return np.mean(np.abs(W[0] - ex)), W


def test_sod_exact_riemann(orc):
    """Sec. 5.2 (b): the oracle converges to the exact Sod solution."""
    e = {n: sod_l1(orc, n)[0] for n in (100, 200, 400)}
    assert e[400] < 2.5e-3, e
    assert e[100] > e[200] > e[400]
    order = math.log2(e[100] / e[400]) / 2
    assert 0.6 < order < 1.3, (e, order)


def test_sod_positivity_and_bounds(orc):
    _, W = sod_l1(orc, 400)
    rho, vel, p = I.primitive(W)
    assert rho.min() > 0.1 and p.min() > 0.09
    assert rho.max() < 1.0 + 1e-3 and p.max() < 1.0 + 1e-3


def periodic_field(nx, ny, seed=0):
    rng = np.random.default_rng(seed)
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y)
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * (X + 2 * Y)) + 0.05 * rng.normal(size=X.shape)
    u = 0.3 + 0.2 * np.cos(2 * np.pi * Y)
    v = -0.2 + 0.1 * np.sin(2 * np.pi * X)
    p = 1.0 + 0.1 * np.cos(2 * np.pi * (X - Y))
    return I.conservative(rho, [u, v], p)


def test_conservation_periodic(orc):
    W = periodic_field(17, 13)
    P = orc.make_params([17, 13], [1 / 17, 1 / 13], bc="periodic")
    dt = orc.cfl_dt(P, W, 0.5)
    tot0 = W.reshape(4, -1).sum(axis=1)
    for _ in range(3):
        W, _, _, bad = orc.step(P, W, dt)
        assert bad == 0
    tot = W.reshape(4, -1).sum(axis=1)
    scale = np.abs(W).reshape(4, -1).sum(axis=1)
    assert np.all(np.abs(tot - tot0) <= 1e-13 * scale), (tot - tot0) / scale


def test_free_stream_preservation(orc):
    W = I.conservative(np.full((9, 11), 0.7), [np.full((9, 11), 0.4), np.full((9, 11), -0.9)], np.full((9, 11), 2.3))
    for bc in ("periodic", "transmissive"):
        P = orc.make_params([11, 9], [0.1, 0.13], bc=bc)
        Wn = W
        for _ in range(5):
            Wn, _, _, bad = orc.step(P, Wn, 0.004)
        np.testing.assert_allclose(Wn, W, rtol=2e-14, atol=0)


def test_transpose_symmetry_2d(orc):
    """x <-> y with U <-> V gives the transposed result (Sec. 3.2 procedure is
    the same in both directions)."""
    W = periodic_field(12, 12, seed=1)
    WT = np.stack([W[0].T, W[2].T, W[1].T, W[3].T])
    P = orc.make_params([12, 12], [1 / 12, 1 / 12], bc="transmissive")
    a, fa, _, _ = orc.step(P, W, 0.01, want_flags=True)
    b, fb, _, _ = orc.step(P, WT, 0.01, want_flags=True)
    bT = np.stack([b[0].T, b[2].T, b[1].T, b[3].T])
    np.testing.assert_allclose(a, bT, rtol=1e-14, atol=1e-15)
    # normal flags of x-sweep on W equal those of the y-sweep on W^T
    n = 12 * 12
    fa_n = fa[: 2 * 4 * n].reshape(2, 4, 12, 12)
    fb_n = fb[: 2 * 4 * n].reshape(2, 4, 12, 12)
    comp = [0, 2, 1, 3]
    for c in range(4):
        assert np.array_equal(fa_n[0, c], fb_n[1, comp[c]].T)


def test_mirror_symmetry_1d(orc):
    W, dx = I.riemann_1d(64, (1.0, 0.3, 1.0), (0.3, -0.2, 0.4))
    Wm = np.stack([W[0][::-1], -W[1][::-1], W[2][::-1]])
    P = orc.make_params([64], [dx], bc="transmissive")
    a, _, _, _ = orc.step(P, W, 0.002)
    b, _, _, _ = orc.step(P, Wm, 0.002)
    np.testing.assert_allclose(a, np.stack([b[0][::-1], -b[1][::-1], b[2][::-1]]), rtol=1e-13, atol=1e-14)


def test_cyclic_symmetry_3d(orc):
    rng = np.random.default_rng(3)
    n = 6
    x = (np.arange(n) + 0.5) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    rho = 1 + 0.2 * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y) + 0.1 * np.sin(2 * np.pi * Z)
    u = 0.2 * np.cos(2 * np.pi * Y)
    v = 0.1 * np.sin(2 * np.pi * Z)
    w = -0.3 * np.cos(2 * np.pi * X)
    p = 1 + 0.05 * rng.normal(size=X.shape)
    W = I.conservative(rho, [u, v, w], p)
    # cyclic map (x, y, z) -> (y, z, x): new[z][y][x] = old at x'=y... realised
    # by moving array axes and rotating velocity components
    def cyc(F):
        return np.stack([np.moveaxis(F[c], [0, 1, 2], [1, 2, 0]) for c in range(5)])[[0, 2, 3, 1, 4]]
    P = orc.make_params([n, n, n], [1 / n] * 3, bc="periodic")
    a, _, _, _ = orc.step(P, W, 0.01)
    b, _, _, _ = orc.step(P, cyc(W), 0.01)
    np.testing.assert_allclose(cyc(a), b, rtol=1e-13, atol=1e-14)


def test_reflective_wall_symmetric_problem(orc):
    # a problem symmetric about x = 1/2 stays symmetric with reflective walls
    n = 40
    x = (np.arange(n) + 0.5) / n
    rho = 1 + 0.5 * np.exp(-50 * (x - 0.5) ** 2)
    W = I.conservative(rho, [0.3 * np.sin(2 * np.pi * x)], 1 + 0.2 * np.cos(2 * np.pi * x))
    P = orc.make_params([n], [1 / n], bc="reflective")
    Wn, _, _, _ = orc.run(P, W, 10, cfl=0.5)
    np.testing.assert_allclose(Wn[0], Wn[0][::-1], rtol=1e-12)
    np.testing.assert_allclose(Wn[1], -Wn[1][::-1], rtol=1e-12, atol=1e-13)
    # total mass conserved with walls
    assert abs(Wn[0].sum() - W[0].sum()) < 1e-12 * W[0].sum()


def amplitude(f, x, k):
    return 2 * np.mean(f * np.sin(k * x))


def test_ns_shear_wave_decay(orc):
    """Linearised Navier-Stokes: v = A sin(kx) decays as exp(-nu k^2 t)."""
    n, mu, A = 32, 0.01, 1e-3
    x = (np.arange(n) + 0.5) / n
    k = 2 * np.pi
    cellavg_sin = (np.cos(k * (x - 0.5 / n)) - np.cos(k * (x + 0.5 / n))) / (k / n)
    v = np.tile(A * cellavg_sin, (3, 1))
    W = I.conservative(np.ones((3, n)), [np.zeros((3, n)), v], np.ones((3, n)))
    P = orc.make_params([n, 3], [1 / n, 1 / 3], bc="periodic", tau="viscous", mu=mu, prandtl=0.72)
    T = 0.2
    Wn, t, s, bad = orc.run(P, W, 10000, cfl=0.5, t_end=T)
    ratio = amplitude(Wn[2][1], x, k) / amplitude(W[2][1], x, k)
    assert abs(ratio / math.exp(-mu * k * k * T) - 1) < 3e-3, ratio


def linear_ns_density(pr, mu, k, T, cv=2.5, KD=5):
    """Density response of the linearised Navier-Stokes equations about
    (rho, u, p) = (1, 0, 1) to an isobaric perturbation rho' = -T' = 1: the
    3x3 Fourier system (continuity, momentum with the BGK normal stress
    2 mu (1 - 1/(K+D)) u_x, energy with conductivity c_p mu / Pr) solved by
    its eigen-decomposition."""
    kap = (cv + 1) * mu / pr
    nu = 2 * mu * (1 - 1 / KD)
    A = np.array([[0, -1j * k, 0], [-1j * k, -nu * k * k, -1j * k], [0, -1j * k / cv, -kap / cv * k * k]])
    ev, V = np.linalg.eig(A)
    c = np.linalg.solve(V, np.array([1, 0, -1]))
    return (V @ (c * np.exp(ev * T)))[0].real


def test_ns_entropy_wave_prandtl(orc):
    """Isobaric temperature perturbation: its decay is set by the heat
    conductivity c_p mu / Pr, so it pins the Prandtl-number correction of the
    energy flux against linearised Navier-Stokes theory."""
    n, mu, pr, eps = 64, 0.01, 0.72, 1e-3
    x = (np.arange(n) + 0.5) / n
    k = 2 * np.pi
    rho = 1 + eps * (np.cos(k * (x - 0.5 / n)) - np.cos(k * (x + 0.5 / n))) / (k / n)
    W = I.conservative(np.tile(rho, (3, 1)), [np.zeros((3, n)), np.zeros((3, n))], np.ones((3, n)))
    P = orc.make_params([n, 3], [1 / n, 1 / 3], bc="periodic", tau="viscous", mu=mu, prandtl=pr)
    T = 0.2
    Wn, t, s, bad = orc.run(P, W, 10000, cfl=0.5, t_end=T)
    ratio = amplitude(Wn[0][1] - 1, x, k) / amplitude(rho - 1, x, k)
    want = linear_ns_density(pr, mu, k, T)
    assert abs(ratio / want - 1) < 1.5e-3, (ratio, want)
    # clearly closer to the Pr = 0.72 response than to the Pr = 1 response
    other = linear_ns_density(1.0, mu, k, T)
    assert abs(ratio - want) < 0.2 * abs(ratio - other)


def test_dual_matches_finite_differences(orc):
    rng = np.random.default_rng(9)
    W = periodic_field(10, 8, seed=4)
    V = np.zeros_like(W)
    V[0] = rng.normal(size=W[0].shape) * 0.1
    P = orc.make_params([10, 8], [0.1, 0.125], bc="periodic")
    dt = 0.01
    _, dW, _ = orc.step_dual(P, W, V, dt)
    h = 1e-6
    Wp, _, _, _ = orc.step(P, W + h * V, dt)
    Wm, _, _, _ = orc.step(P, W - h * V, dt)
    fd = (Wp - Wm) / (2 * h)
    assert np.abs(fd - dW).max() <= 1e-6 * np.abs(dW).max()


def test_step_failure_count_and_invalid_args(orc):
    W, dx = I.sod(32)
    W = W.copy()
    W[2, 5] = -1.0  # negative energy in one cell
    P = orc.make_params([32], [dx])
    _, _, _, bad = orc.step(P, W, 1e-3)
    assert bad > 0
    with pytest.raises(ValueError):
        orc.step(P, W, -1.0)
    Pbad = orc.make_params([2], [dx])
    with pytest.raises(ValueError):
        orc.step(Pbad, W[:, :2], 1e-3)


def test_cfl_time_step(orc):
    W, dx = I.sod(10)
    P = orc.make_params([10], [dx])
    # max over cells of |U| + a is the sound speed of the left state, sqrt(1.4)
    assert abs(orc.cfl_dt(P, W, 0.5) - 0.5 * dx / math.sqrt(1.4)) < 1e-15
    Pv = orc.make_params([10], [dx], mu=1.0, tau="viscous")
    assert abs(orc.cfl_dt(Pv, W, 0.5) - 0.5 * dx * dx * 0.125 / 4.0) < 1e-15
