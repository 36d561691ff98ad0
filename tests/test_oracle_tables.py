"""Pins of the oracle against the error tables the paper prints for TENO-D GKS.

Table 4 (Sec. 5.1, 1-D density wave) and Table 8 (Sec. 5.5, 2-D density wave)
are reproduced to 6-7 significant digits.  They pin, end to end, the
large-stencil reconstruction (Eqs. 4.8-4.9), the kinetic weighting of the
equilibrium state (Eq. 2.6), the tau = 0 flux with its time derivative
(Eqs. 2.5-2.9), the S2O4 update (Sec. 2.2), the tangential Gauss-point
reconstruction (Sec. 3.2 Steps 1-3) and the CFL step (Sec. 5).

Readings fixed by these tables:
  * 1-D: the table is reproduced with CFL 0.5 time steps; the fixed
    dt = 0.2 dx printed in the caption gives errors 0.65 % higher.
  * 1-D "mesh length" is the cell width (n = 2/h); 2-D "mesh length" is 1/n.
  * errors are mean / rms / max over cells against exact cell averages.
"""
import os

import numpy as np
import pytest

from paper_2309_10534_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    rows = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t = line.split()
            rows[int(t[0])] = np.array([float(x) for x in t[2:5]])
    return rows


def errors(W, exact):
    e = W[0] - exact[0]
    return np.array([np.mean(np.abs(e)), np.sqrt(np.mean(e * e)), np.max(np.abs(e))])


TABLE4 = load("table4_teno_d_density_wave_1d.txt")
TABLE8 = load("table8_teno_d_density_wave_2d.txt")


def run_1d(orc, n, **kw):
    W0, dx = I.density_wave_1d(n)
    P = orc.make_params([n], [dx], bc="periodic", tau="zero")
    W, t, s, bad = orc.run(P, W0, 100000, t_end=2.0, **kw)
    assert bad == 0 and abs(t - 2.0) < 1e-12
    ex, _ = I.density_wave_1d(n, t=2.0)
    return errors(W, ex)


@pytest.mark.parametrize("n", [10, 20, 40, 80, 160])
def test_table4_1d_density_wave(orc, n):
    err = run_1d(orc, n, cfl=0.5)
    tol = 5e-3 if n == 10 else 2e-5
    np.testing.assert_allclose(err, TABLE4[n], rtol=tol)


def test_table4_orders(orc):
    errs = [run_1d(orc, n, cfl=0.5)[0] for n in (20, 40, 80, 160)]
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - 5.0) < 0.03), orders


def test_table4_caption_dt_reading(orc):
    # The fixed dt = 0.2 dx of the caption reproduces the table only to ~0.7 %.
    n = 40
    W0, dx = I.density_wave_1d(n)
    P = orc.make_params([n], [dx], bc="periodic", tau="zero")
    dt = 0.2 * dx
    W, t, s, bad = orc.run(P, W0, int(round(2.0 / dt)), fixed_dt=dt)
    ex, _ = I.density_wave_1d(n, t=2.0)
    ratio = errors(W, ex)[0] / TABLE4[n][0]
    assert 1.003 < ratio < 1.01


def run_2d(orc, n):
    W0, dx = I.density_wave_2d(n)
    P = orc.make_params([n, n], [dx, dx], bc="periodic", tau="zero")
    W, t, s, bad = orc.run(P, W0, 100000, cfl=0.5, t_end=2.0)
    assert bad == 0 and abs(t - 2.0) < 1e-12
    ex, _ = I.density_wave_2d(n, t=2.0)
    return errors(W, ex)


@pytest.mark.parametrize("n", [5, 10, 20, 40])
def test_table8_2d_density_wave(orc, n):
    err = run_2d(orc, n)
    # the 5-cell periodic grid (stencils wrap around the domain) agrees to 10 %
    tol = {5: 0.12, 10: 1e-5, 20: 1e-5, 40: 1e-5}[n]
    np.testing.assert_allclose(err, TABLE8[n], rtol=tol)


@pytest.mark.skipif(not os.environ.get("TGKS_SLOW"), reason="about 3 min on 8 cores; set TGKS_SLOW=1")
def test_table8_2d_density_wave_n80(orc):
    np.testing.assert_allclose(run_2d(orc, 80), TABLE8[80], rtol=1e-5)
