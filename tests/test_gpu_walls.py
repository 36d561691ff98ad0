"""GPU parity of the no-slip adiabatic wall (Sec. 5.8) against the oracle:
one step on identical input (1e-10, selection flags bit for bit) in 1-D,
2-D (the viscous shock tube's walls and symmetry line) and 3-D, mass and
energy of a closed box kept by the device path (the reverse mode with
walls is checked with the other reverse-mode tests)."""
import numpy as np
import pytest

from gpu_common import GpuProblem, close_scaled, orc_params, problem
from paper_2309_10534_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def compare_step(orc, pr, W, dt, tol=1e-10):
    gp = GpuProblem(pr)
    try:
        print(f"[wall] step shape={pr['shape']} bc={pr['bc']}", flush=True)
        Wg, Wsg, fg, badg = gp.step(W, dt, flags=True)
    finally:
        gp.close()
    Wo, fo, Wso, bado = orc.step(orc_params(orc, pr), W, dt, want_flags=True, want_wstar=True)
    assert np.all(np.isfinite(Wo))
    close_scaled(Wsg, Wso, tol, "W*")
    close_scaled(Wg, Wo, tol, "W^{n+1}")
    assert badg == bado
    mism = np.flatnonzero(fg != fo)
    assert mism.size == 0, f"{mism.size} flag mismatches, first at {mism[:10]}"
    return Wg


def box_state(shape, seed):
    rng = np.random.default_rng(seed)
    sh = tuple(reversed(shape))
    grids = np.meshgrid(*[(np.arange(n) + 0.5) / n for n in reversed(shape)], indexing="ij")
    phase = sum((k + 1) * g for k, g in enumerate(grids))
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * phase) + 0.01 * rng.normal(size=sh)
    vel = [0.2 * np.cos(2 * np.pi * (phase + 0.3 * k)) for k in range(len(shape))]
    p = 1.0 + 0.1 * np.cos(2 * np.pi * phase)
    return I.conservative(rho, vel, p)


@pytest.mark.parametrize("shape", [[41], [37, 29], [9, 7, 6]])
def test_closed_box(orc, torch_dev, shape):
    W = box_state(shape, seed=len(shape))
    pr = problem(shape, [1.0 / n for n in shape], bc="noslip", tau="viscous", mu=5e-3, prandtl=0.72)
    Wg = compare_step(orc, pr, W, 0.5 * orc.cfl_dt(orc_params(orc, pr), W, 0.5))
    D = len(shape)
    for c in (0, D + 1):
        assert abs(Wg[c].sum() - W[c].sum()) <= 1e-13 * abs(W[c].sum())


def test_viscous_shock_tube_walls(orc, torch_dev):
    """The boundary set of the viscous shock tube: no-slip walls left, right
    and at the bottom, symmetry (reflective) at the top; its initial data on
    a small grid, a few steps in characteristic variables (with conservative
    variables the 100:1 membrane drives the scheme, which has no positivity
    limiter, to negative states in the second step)."""
    W, dx = I.viscous_shock_tube(40, 20)
    pr = problem([40, 20], [dx, dx], bc=[("noslip", "noslip"), ("noslip", "reflective")], tau="viscous",
                 mu=1.0 / 200.0, prandtl=0.73, recon=1)
    P = orc_params(orc, pr)
    for _ in range(3):
        W = compare_step(orc, pr, W, orc.cfl_dt(P, W, 0.2))


def test_euler_walls_and_characteristic(orc, torch_dev):
    W = box_state([33, 17], seed=5)
    pr = problem([33, 17], [1 / 33, 1 / 17], bc=[("noslip", "transmissive"), ("periodic", "periodic")], recon=1)
    compare_step(orc, pr, W, 0.5 * orc.cfl_dt(orc_params(orc, pr), W, 0.5))
