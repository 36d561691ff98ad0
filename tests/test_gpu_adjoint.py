"""Reverse mode on the GPU: tgks_step_adjoint and the checkpointed rollout.

One step: <G, J V> with J V the oracle's forward-mode derivative of its own
step (dual numbers; stencil selections taken on the primal values, dt
constant) against <J^T G, V> from the HIP reverse kernels, relative to
sum |G * J V|, bar 1e-10.  Rollouts: the same over several steps with the
oracle's own CFL steps fed to both sides, and central differences of the
HIP forward along seeded smooth directions at the full 512 x 512 vortex."""
import numpy as np
import pytest

from gpu_common import GpuProblem, orc_params, problem
from paper_2309_10534_amd import inputs as I

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def smooth_field(shape, seed, amp=0.2):
    """Smooth positive state on a (possibly ragged) grid: sums of low modes."""
    rng = np.random.default_rng(seed)
    D = len(shape)
    axes = np.meshgrid(*[np.arange(n) / n for n in shape[::-1]], indexing="ij")[::-1]

    def mode():
        out = 0.0
        for k in range(1, 3):
            for x in axes:
                out = out + rng.uniform(-1, 1) * np.sin(2 * np.pi * k * x + rng.uniform(0, 2 * np.pi))
        return out

    rho = 1.0 + amp * 0.5 * mode()
    vel = [0.3 * rng.uniform(-1, 1) + amp * 0.5 * mode() for _ in range(D)]
    p = 1.0 + amp * 0.5 * mode()
    return I.conservative(rho, vel, p)


def adjoint_vs_oracle(orc, torch, pr, W, dt, seed=0):
    from paper_2309_10534_amd import tgks
    rng = np.random.default_rng(seed)
    G = rng.standard_normal(W.shape)
    V = rng.standard_normal(W.shape)
    gp = GpuProblem(pr)
    try:
        print(f"[adjoint] step shape={pr['shape']} bc={pr['bc']} tau={pr['tau']} mu={pr['mu']}", flush=True)
        Wd, Gd = gp.dev(W), gp.dev(G)
        out = torch.empty_like(Gd)
        dtd = torch.tensor([dt], dtype=torch.float64, device="cuda")
        tgks.tgks_step_adjoint(gp.ctx, Wd, dtd, Gd, out)
        torch.cuda.synchronize()
        Gin = out.cpu().numpy().reshape(W.shape)
        # with the step's W* handed in: the same cotangent, bit for bit
        Wn, Ws = torch.empty_like(Wd), torch.empty_like(Wd)
        tgks.tgks_step(gp.ctx, Wd, Wn, dtd, None, Ws)
        out2 = torch.empty_like(Gd)
        tgks.tgks_step_adjoint(gp.ctx, Wd, dtd, Gd, out2, W_star=Ws)
        torch.cuda.synchronize()
        assert torch.equal(out, out2)
    finally:
        gp.close()
    Wo, dWo, bad = orc.step_dual(orc_params(orc, pr), W, V, dt)
    assert bad == 0 and np.all(np.isfinite(Wo))
    lhs = float(np.sum(G * dWo))
    rhs = float(np.sum(Gin * V))
    scale = float(np.sum(np.abs(G * dWo)))
    assert abs(lhs - rhs) <= TOL * scale, f"<G,JV>={lhs!r} <J^T G,V>={rhs!r} rel {abs(lhs - rhs) / scale:.2e}"
    return Gin


@pytest.mark.parametrize("bc", ["periodic", "transmissive", "reflective", "noslip",
                                [("noslip", "noslip"), ("noslip", "reflective")]])
def test_step_adjoint_2d_smooth_ragged(orc, torch_dev, bc):
    shape = [37, 29]  # several 8 x 16 face tiles with ragged tails
    W = smooth_field(shape, seed=3)
    pr = problem(shape, [0.1, 0.13], bc=bc)
    dt = orc.cfl_dt(orc_params(orc, pr), W, 0.5)
    adjoint_vs_oracle(orc, torch_dev, pr, W, dt, seed=1)


def test_step_adjoint_2d_discontinuous(orc, torch_dev):
    """A smooth field with a slanted jump in density and pressure: the
    small-stencil selections near the jump, the large stencil elsewhere.
    (Piecewise-constant data is not used here: in a constant region every
    selection of the intermediate state W* is decided by rounding residues of
    order 1e-30, which differ between two correct evaluations of W*, and the
    derivative with frozen selections depends on them even though the values
    do not.)"""
    shape = [34, 30]
    W = smooth_field(shape, seed=21, amp=0.1)
    ny, nx = shape[1], shape[0]
    y, x = np.meshgrid((np.arange(ny) + 0.5) / ny, (np.arange(nx) + 0.5) / nx, indexing="ij")
    jump = x + 0.6 * y > 0.7
    rho, vel, p = I.primitive(W)
    W = I.conservative(rho * np.where(jump, 2.0, 1.0), vel, p * np.where(jump, 1.8, 1.0))
    pr = problem(shape, [1 / nx, 1 / ny])
    dt = orc.cfl_dt(orc_params(orc, pr), W, 0.5)
    adjoint_vs_oracle(orc, torch_dev, pr, W, dt, seed=2)


def test_step_adjoint_2d_navier_stokes(orc, torch_dev):
    shape = [24, 20]
    W = smooth_field(shape, seed=5)
    pr = problem(shape, [0.05, 0.05], bc="periodic", tau="viscous", mu=2e-3, prandtl=0.72)
    dt = orc.cfl_dt(orc_params(orc, pr), W, 0.4)
    adjoint_vs_oracle(orc, torch_dev, pr, W, dt, seed=3)


def test_step_adjoint_2d_vortex(orc, torch_dev):
    """The strength-5 vortex, off the centre of the cells' symmetry lines.
    (Centred, the normal slopes of rho and of the normal momentum vanish on
    the vortex's symmetry lines up to rounding, the tangential selections of
    those slopes are decided by rounding, and the frozen-selection
    derivatives of two correct implementations differ there: measured 1.8e-6
    relative at 32 x 32.)"""
    W, dx = I.isentropic_vortex_2d(32, center=(4.83, 5.27))
    pr = problem([32, 32], [dx, dx], bc="periodic")
    dt = orc.cfl_dt(orc_params(orc, pr), W, 0.5)
    adjoint_vs_oracle(orc, torch_dev, pr, W, dt, seed=4)


@pytest.mark.parametrize("case", ["sod", "wave", "reflective", "viscous", "noslip"])
def test_step_adjoint_1d(orc, torch_dev, case):
    if case == "sod":
        # Sod's states with a smooth modulation (no exactly constant region)
        W, dx = I.sod(120)
        x = (np.arange(120) + 0.5) / 120
        rho, vel, p = I.primitive(W)
        W = I.conservative(rho * (1 + 0.05 * np.sin(2 * np.pi * x)), vel, p * (1 + 0.05 * np.cos(2 * np.pi * x)))
        pr = problem([120], [dx])
    elif case == "wave":
        # the density wave with a pressure modulation: at uniform pressure the
        # sign of p_l - p_r in the collision time is decided by rounding, and
        # the derivative of |p_l - p_r| with it
        W, dx = I.density_wave_1d(50)
        x = (np.arange(50) + 0.5) / 50
        rho, vel, p = I.primitive(W)
        W = I.conservative(rho, vel, p * (1 + 0.1 * np.cos(2 * np.pi * x)))
        pr = problem([50], [dx], bc="periodic")
    elif case == "reflective":
        W = smooth_field([90], seed=8)
        dx = 1 / 90
        pr = problem([90], [dx], bc=[("reflective", "reflective")])
    elif case == "noslip":
        W = smooth_field([90], seed=9)
        dx = 1 / 90
        pr = problem([90], [dx], bc=[("noslip", "transmissive")], tau="viscous", mu=2e-3, prandtl=0.72)
    else:
        W = smooth_field([64], seed=9)
        pr = problem([64], [1 / 64], bc="periodic", tau="viscous", mu=1e-3, prandtl=0.72)
    dt = orc.cfl_dt(orc_params(orc, pr), W, 0.5)
    adjoint_vs_oracle(orc, torch_dev, pr, W, dt, seed=5)


def test_step_adjoint_invalid(torch_dev):
    from paper_2309_10534_amd import tgks
    gp = GpuProblem(problem([8, 8, 8], [0.1] * 3))
    try:
        W = torch_dev.ones(gp.n, dtype=torch_dev.float64, device="cuda")
        dt = torch_dev.ones(1, dtype=torch_dev.float64, device="cuda")
        with pytest.raises(tgks.TgksError):
            tgks.tgks_step_adjoint(gp.ctx, W, dt, W.clone(), W.clone())
    finally:
        gp.close()
    gp = GpuProblem(problem([16, 16], [0.1] * 2))
    try:
        W = torch_dev.ones(gp.n, dtype=torch_dev.float64, device="cuda")
        dt = torch_dev.ones(1, dtype=torch_dev.float64, device="cuda")
        with pytest.raises(tgks.TgksError):
            tgks.tgks_step_adjoint(gp.ctx, W, dt, W, W)  # output aliases the input cotangent
    finally:
        gp.close()


def test_rollout_adjoint_vs_oracle_chain(orc, torch_dev):
    """8 steps, checkpoints every 3 (a partial last segment): the reverse of
    the rollout against the oracle's forward-mode derivative carried through
    the same 8 steps (the oracle's own CFL steps, fed to both sides)."""
    from paper_2309_10534_amd import tgks
    from paper_2309_10534_amd.rollout import rollout, rollout_adjoint
    torch = torch_dev
    shape = [26, 22]
    W0 = smooth_field(shape, seed=11)
    pr = problem(shape, [0.08, 0.08], bc="periodic")
    P = orc_params(orc, pr)
    rng = np.random.default_rng(12)
    V = rng.standard_normal(W0.shape)
    G = rng.standard_normal(W0.shape)
    W, dW, dts = W0.copy(), V.copy(), []
    for _ in range(8):
        dt = orc.cfl_dt(P, W, 0.5)
        dts.append(dt)
        W, dW, bad = orc.step_dual(P, W, dW, dt)
        assert bad == 0
    lhs = float(np.sum(G * dW))
    gp = GpuProblem(pr)
    try:
        dtd = torch.tensor(dts, dtype=torch.float64, device="cuda")
        Wn, _, ck = rollout(gp.ctx, gp.dev(W0), 8, dts=dtd, every=3)
        g0 = rollout_adjoint(gp.ctx, ck, dtd, gp.dev(G), every=3)
        torch.cuda.synchronize()
        rhs = float(np.sum(g0.cpu().numpy().reshape(W0.shape) * V))
        assert np.abs(Wn.cpu().numpy().reshape(W0.shape) - W).max() < 1e-12 * np.abs(W).max()
    finally:
        gp.close()
    scale = float(np.sum(np.abs(G * dW)))
    assert abs(lhs - rhs) <= TOL * scale, (lhs, rhs)


def density_directions(n, seeds, kmax=8):
    """Smooth directions in the density component: random Fourier modes with
    |k| <= kmax on the periodic grid, one per seed."""
    out = []
    x = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(x, x, indexing="xy")
    for s in seeds:
        rng = np.random.default_rng(s)
        v = np.zeros((n, n))
        for kx in range(-kmax, kmax + 1):
            for ky in range(0, kmax + 1):
                if kx * kx + ky * ky == 0 or kx * kx + ky * ky > kmax * kmax:
                    continue
                v += rng.standard_normal() * np.cos(2 * np.pi * (kx * X + ky * Y) + rng.uniform(0, 2 * np.pi))
        out.append(v / np.abs(v).max())
    return out


def test_rollout_autograd_fd_vortex_512(torch_dev):
    """Full size: 2-D isentropic vortex (strength 5, mean flow (1, 1)) on
    512 x 512 periodic cells of [0, 10]^2, 200 steps at CFL 0.5, checkpoints
    every 20; J = dx dy sum rho^2 at the final time; gradient with respect to
    the initial density against central differences of the forward (the
    recorded steps fixed) along seeded smooth directions."""
    from paper_2309_10534_amd import tgks
    from paper_2309_10534_amd.rollout import GKSRollout, rollout
    torch = torch_dev
    n, steps = 512, 200
    W0, dx = I.isentropic_vortex_2d(n)
    pr = problem([n, n], [dx, dx], bc="periodic")
    gp = GpuProblem(pr)
    try:
        print(f"[adjoint] vortex {n}^2 {steps} steps", flush=True)
        W0d = gp.dev(W0).requires_grad_(True)
        Wn = GKSRollout.apply(W0d, gp.ctx, steps, 0.5, 20)
        J = (Wn[0] ** 2).sum() * dx * dx
        (g,) = torch.autograd.grad(J, W0d)
        assert tgks.tgks_status(gp.ctx) == 0
        _, dts, _ = rollout(gp.ctx, gp.dev(W0), steps, 0.5, every=steps + 1)
        gr = g[0].double()
        for v in density_directions(n, range(10, 15)):
            eps = 1e-6
            vd = torch.from_numpy(v).cuda()

            def J_of(s):
                W = gp.dev(W0)
                W[0] += s * vd
                Wf, _, _ = rollout(gp.ctx, W, steps, dts=dts, every=steps + 1)
                return float((Wf[0] ** 2).sum() * dx * dx)

            fd = (J_of(eps) - J_of(-eps)) / (2 * eps)
            ad = float((gr * vd).sum())
            print(f"[adjoint] direction: adjoint {ad:.12e} fd {fd:.12e} rel {abs(ad - fd) / abs(fd):.2e}",
                  flush=True)
            assert abs(ad - fd) <= 1e-6 * abs(fd)
    finally:
        gp.close()
