"""GPU parity of the optional first-order fallback at non-physical
Gauss-point states against the oracle.  Each step starts from a state on
the oracle's own trajectory, so that both sides decide on the same input:
the double Mach reflection (Sec. 5.7) at steps 0, 10 and 25 (its first step
has non-physical states at the shock foot) and a periodic blast, 1e-10
L1-relative with selection flags bit for bit and the same number of
replaced Gauss-point states; the device run of the blast keeps mass,
momentum and energy."""
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


def compare_on_trajectory(orc, pr, W0, marks, t_of=None):
    P = orc_params(orc, pr)
    W, t, k = W0.copy(), 0.0, 0
    counts = []
    gp = GpuProblem(pr)
    try:
        while k <= max(marks):
            dt = orc.cfl_dt(P, W, 0.5)
            if k in marks:
                print(f"[fallback] shape={pr['shape']} recon={pr.get('recon', 0)} step={k}", flush=True)
                Wg, Wsg, fg, badg = gp.step(W, dt, flags=True, t0=t)
                nfb = [0]
                Wo, fo, Wso, bado = orc.step(P, W, dt, want_flags=True, want_wstar=True, t=t, fallbacks=nfb)
                assert badg == bado == 0
                assert gp.fallbacks == nfb[0], (gp.fallbacks, nfb[0])  # the same decisions
                counts.append(nfb[0])
                mism = np.flatnonzero(fg != fo)
                assert mism.size == 0, f"{mism.size} flag mismatches, first at {mism[:10]}"
                close_scaled(Wsg, Wso, 1e-10, f"W* step {k}")
                close_scaled(Wg, Wo, 1e-10, f"W^(n+1) step {k}")
                W = Wo
            else:
                W = orc.step(P, W, dt, t=t)[0]
            t += dt
            k += 1
    finally:
        gp.close()
    return counts


@pytest.mark.parametrize("recon", [0, 1])
def test_double_mach_steps(orc, torch_dev, recon):
    W0, (dx, dy), spec = I.double_mach(96, 24)
    pr = problem([96, 24], [dx, dy], bc=spec["bc"], states=spec["states"], lines=spec["lines"], far=spec["far"],
                 recon=recon, fallback=1)
    counts = compare_on_trajectory(orc, pr, W0, (0, 10, 25))
    assert counts[0] > 0  # the first step needs the fallback


def blast(n):
    x = (np.arange(n) + 0.5) / n
    p = np.where(x < 0.1, 1000.0, np.where(x > 0.9, 100.0, 0.01))
    return I.conservative(np.ones(n), [np.zeros(n)], p), 1.0 / n


@pytest.mark.parametrize("recon", [0, 1])
def test_periodic_blast(orc, torch_dev, recon):
    W0, dx = blast(203)
    pr = problem([203], [dx], bc="periodic", recon=recon, fallback=1)
    compare_on_trajectory(orc, pr, W0, (0, 3, 20))
    gp = GpuProblem(pr)
    try:
        print(f"[fallback] blast run recon={recon}", flush=True)
        W, td, bad = gp.run(W0, 300, cfl=0.5)
    finally:
        gp.close()
    assert bad == 0 and np.all(np.isfinite(W))
    for c in range(3):
        scale = np.abs(W0[c]).sum() + np.abs(W0[2]).sum() * (c == 1)
        assert abs(W[c].sum() - W0[c].sum()) <= 1e-13 * scale, c


def test_rejections(torch_dev):
    from paper_2309_10534_amd import tgks
    p1 = tgks.tgks_params_default(2, [16, 16], [0.1, 0.1], fallback=1)
    p0 = tgks.tgks_params_default(2, [16, 16], [0.1, 0.1])
    with pytest.raises(tgks.TgksError):  # mixed within one batch
        tgks.tgks_batch_create([p1, p0])


def blast_3d(nx=20, n=6):
    """Periodic 3-D tube along x: density 1 / 1e-3 across x = 1/2, pressure
    1e4 for x < 0.15 and 1e-3 elsewhere (the fallback acts in the first
    steps); every face direction is exercised."""
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(n) + 0.5) / n
    Z, Y, X = np.meshgrid(y, y, x, indexing="ij")
    rho = np.where(X < 0.5, 1.0, 1e-3)
    p = np.where(X < 0.15, 1e4, 1e-3)
    return I.conservative(rho, [np.zeros_like(rho)] * 3, p), [1.0 / nx, 1.0 / n, 1.0 / n]


def test_tube_3d(orc, torch_dev):
    """3-D: steps 0, 1, 3 and 6 along the oracle's trajectory (the fallback
    acts in the first three) agree: 1e-10, flags bit for bit, the same
    number of replaced states."""
    W0, dx = blast_3d()
    pr = problem([20, 6, 6], dx, bc="periodic", fallback=1)
    counts = compare_on_trajectory(orc, pr, W0, (0, 1, 3, 6))
    assert counts[0] > 0 and counts[1] > 0
