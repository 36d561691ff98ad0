"""GPU parity of the prescribed sides (the inflow, post-shock bottom and
moving-shock top of the double Mach reflection, Sec. 5.7) against the
oracle: single steps from a non-zero time (1e-10 L1-relative, selection
flags bit for bit, tile rows ragged), CFL runs from a non-zero time origin
eagerly and from a graph, the 1-D inflow shock, the double Mach reflection's
own first step (non-physical Gauss-point states included: same count, same
cells), and the contexts that reject prescribed sides."""
import math

import numpy as np
import pytest

from gpu_common import GpuProblem, assert_close, orc_params, problem
from paper_2309_10534_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def shock_post(ms, rho1=1.4, p1=1.0, gamma=1.4):
    m2 = ms * ms
    rho2 = rho1 * (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    p2 = p1 * (2.0 * gamma * m2 - (gamma - 1.0)) / (gamma + 1.0)
    S = ms * math.sqrt(gamma * p1 / rho1)
    return (rho2, S * (1.0 - rho1 / rho2), p2), S


def dmr_like(nx, ny, ms=1.5, recon=0, bottom_far="reflective"):
    """The double Mach reflection's boundary layout around a Mach ms shock."""
    (rho2, un, p2), S = shock_post(ms)
    post = (rho2, un * math.sqrt(3.0) / 2.0, -0.5 * un, p2)
    W, (dx, dy), A, B = I.oblique_shock(nx, ny, post, I.DMR_PRE)
    s3 = math.sqrt(3.0)
    pr = problem([nx, ny], [dx, dy], bc=[("prescribed", "transmissive"), ("prescribed", "prescribed")],
                 recon=recon, states=(A.tolist(), B.tolist()),
                 lines={(0, 0): (math.inf, 0.0, 0.0), (1, 0): (1.0 / 6.0, 0.0, 0.0),
                        (1, 1): (1.0 / 6.0, 1.0 / s3, 2.0 * S / s3)},
                 far={(1, 0): bottom_far, (1, 1): "state_b"})
    return pr, W


def compare_step(orc, pr, W, dt, t0, tol=1e-10):
    gp = GpuProblem(pr)
    try:
        print(f"[prescribed] step shape={pr['shape']} recon={pr.get('recon', 0)} t0={t0}", flush=True)
        Wg, Wsg, fg, badg = gp.step(W, dt, flags=True, t0=t0)
    finally:
        gp.close()
    Wo, fo, Wso, bado = orc.step(orc_params(orc, pr), W, dt, want_flags=True, want_wstar=True, t=t0)
    assert badg == bado
    mism = np.flatnonzero(fg != fo)
    assert mism.size == 0, f"{mism.size} flag mismatches, first at {mism[:10]}"
    return Wg, Wsg, Wo, Wso, bado


@pytest.mark.parametrize("recon", [0, 1])
@pytest.mark.parametrize("bottom_far", ["reflective", "transmissive", "state_b"])
def test_step_dmr_layout(orc, torch_dev, recon, bottom_far):
    """Mach 1.5 shock in the double Mach reflection's layout, 100 x 26 cells
    (ragged tiles along both axes), one step from t0 = 0.013 (the top's
    states depend on it)."""
    pr, W = dmr_like(100, 26, recon=recon, bottom_far=bottom_far)
    dt = orc.cfl_dt(orc_params(orc, pr), W, 0.5)
    Wg, Wsg, Wo, Wso, bad = compare_step(orc, pr, W, dt, 0.013)
    assert bad == 0
    assert_close(Wsg, Wso, what="W*")
    assert_close(Wg, Wo, what="W^{n+1}")


def test_step_time_matters(orc, torch_dev):
    """The same step from two times differs at the top only, on both paths."""
    pr, W = dmr_like(64, 16)
    dt = orc.cfl_dt(orc_params(orc, pr), W, 0.5)
    Wg1 = compare_step(orc, pr, W, dt, 0.0)[0]
    Wg2, _, Wo2, _, _ = compare_step(orc, pr, W, dt, 0.05)
    assert_close(Wg2, Wo2, what="t0 = 0.05")
    diff_rows = np.flatnonzero(np.abs(Wg2 - Wg1).max(axis=(0, 2)) > 0)
    assert diff_rows.size > 0 and diff_rows.min() >= 16 - 7


@pytest.mark.parametrize("use_graph", [False, True])
def test_run_from_time_origin(orc, torch_dev, use_graph):
    """Eight CFL steps from the time origin 0.02 (device clock plus origin),
    eagerly and from a captured graph, then eight more from the first run's
    end with the origin moved there."""
    pr, W = dmr_like(80, 20)
    gp = GpuProblem(pr)
    try:
        print(f"[prescribed] run graph={use_graph}", flush=True)
        Wg, td, badg = gp.run(W, 8, cfl=0.5, use_graph=use_graph, t0=0.02)
        Wg2, td2, badg2 = gp.run(Wg, 8, cfl=0.5, use_graph=use_graph, t0=0.02 + td[0])
    finally:
        gp.close()
    P = orc_params(orc, pr)
    Wo, t, s, bado = orc.run(P, W, 8, cfl=0.5, t0=0.02)
    assert badg == bado == 0 and s == 8
    assert abs(td[0] - t) <= 1e-15 * t
    assert_close(Wg, Wo, what="run")
    Wo2, t2, _, _ = orc.run(P, Wo, 8, cfl=0.5, t0=0.02 + t)
    assert badg2 == 0
    assert_close(Wg2, Wo2, what="second run")


def test_inflow_shock_1d(orc, torch_dev):
    (rho2, u2, p2), S = shock_post(3.0)
    n = 203
    B = I.conservative(np.full(n, 1.4), [np.zeros(n)], np.full(n, 1.0))
    A = I.conservative(np.array(rho2), [np.array(u2)], np.array(p2))
    for recon in (0, 1):
        pr = problem([n], [1.0 / n], bc=[("prescribed", "transmissive")], recon=recon,
                     states=(A.tolist(), [0.0, 0.0, 0.0]), lines={(0, 0): (math.inf, 0.0, 0.0)})
        gp = GpuProblem(pr)
        try:
            print(f"[prescribed] 1-D inflow recon={recon}", flush=True)
            Wg, td, badg = gp.run(B, 30, cfl=0.5)
        finally:
            gp.close()
        Wo, t, s, bado = orc.run(orc_params(orc, pr), B, 30, cfl=0.5)
        assert badg == bado == 0
        assert_close(Wg, Wo, what=f"1-D inflow recon={recon}")
        assert Wo[0].max() > 0.9 * rho2  # the shock has formed


def test_double_mach_first_step(orc, torch_dev):
    """The double Mach reflection itself (Mach 10, 192 x 48): its first step
    produces non-physical Gauss-point states at the shock foot next to the
    slip wall; the device path counts as many as the oracle, its
    non-finite cells are the oracle's, and the finite cells agree."""
    W, (dx, dy), spec = I.double_mach(192, 48)
    pr = problem([192, 48], [dx, dy], bc=spec["bc"], states=spec["states"], lines=spec["lines"],
                 far=spec["far"])
    dt = orc.cfl_dt(orc_params(orc, pr), W, 0.5)
    Wg, Wsg, Wo, Wso, bad = compare_step(orc, pr, W, dt, 0.0)
    assert bad > 0
    for a, b in ((Wsg, Wso), (Wg, Wo)):
        fin = np.isfinite(b)
        assert np.array_equal(np.isfinite(a), fin)
        good = fin.all(axis=0)
        for c in range(4):
            e = np.abs(a[c][good] - b[c][good]).sum() / np.abs(b[c][good]).sum()
            assert e <= 1e-10, (c, e)


def test_rejections(torch_dev):
    from paper_2309_10534_amd import tgks
    p3 = tgks.tgks_params_default(3, [8, 8, 8], [0.1] * 3, [("prescribed", "transmissive")] * 3)
    with pytest.raises(tgks.TgksError):
        tgks.tgks_create(p3)
    pr, W = dmr_like(32, 8)
    from gpu_common import gpu_params
    p2 = gpu_params(pr)
    with pytest.raises(tgks.TgksError):
        tgks.tgks_batch_create([p2, p2])
    p2.bc_far[1][0] = tgks.BC_NOSLIP
    with pytest.raises(tgks.TgksError):
        tgks.tgks_create(p2)
    gp = GpuProblem(pr)
    try:
        import torch
        Wd = gp.dev(W)
        g = torch.zeros_like(Wd)
        dtd = torch.tensor([1e-3], dtype=torch.float64, device="cuda")
        with pytest.raises(tgks.TgksError):
            tgks.tgks_step_adjoint(gp.ctx, Wd, dtd, g, torch.zeros_like(Wd))
    finally:
        gp.close()


def test_corner_rule(orc, torch_dev):
    """Corner ghost cells where the x and y sides prescribe different states
    (x: A, y: B): the x side decides on both paths.  (Their influence is
    small: the stencil selections avoid the inconsistent corner cells, and
    giving the corners B instead moves the step by 4e-16.)"""
    rng = np.random.default_rng(11)
    nx, ny = 40, 23
    W = I.conservative(1.0 + 0.3 * rng.random((ny, nx)), [0.3 * rng.standard_normal((ny, nx)),
                       0.3 * rng.standard_normal((ny, nx))], 1.0 + 0.3 * rng.random((ny, nx)))
    A = I.conservative(np.array(1.6), [np.array(0.4), np.array(-0.2)], np.array(1.8))
    B = I.conservative(np.array(0.7), [np.array(-0.1), np.array(0.3)], np.array(0.6))
    every, never = (math.inf, 0.0, 0.0), (-math.inf, 0.0, 0.0)
    pr = problem([nx, ny], [1.0 / nx, 1.0 / ny], bc=[("prescribed", "prescribed"), ("prescribed", "prescribed")],
                 states=(A.tolist(), B.tolist()),
                 lines={(0, 0): every, (0, 1): every, (1, 0): never, (1, 1): never},
                 far={(1, 0): "state_b", (1, 1): "state_b"})
    dt = orc.cfl_dt(orc_params(orc, pr), W, 0.5)
    Wg, Wsg, Wo, Wso, bad = compare_step(orc, pr, W, dt, 0.0)
    assert bad == 0
    assert_close(Wg, Wo, what="corner rule")


def test_state_switch_inside_a_step(orc, torch_dev):
    """1-D: the left side switches from B to A at t = 0.01 (s0 = -0.01,
    s_t = 1); a step from just before, whose stage 2 (at t + dt/2) sees A
    while stage 1 sees B, and steps on either side of it."""
    n = 64
    rng = np.random.default_rng(3)
    W = I.conservative(1.0 + 0.2 * rng.random(n), [0.2 * rng.standard_normal(n)], 1.0 + 0.2 * rng.random(n))
    A = I.conservative(np.array(1.5), [np.array(0.5)], np.array(1.4))
    B = I.conservative(np.array(0.8), [np.array(-0.2)], np.array(0.7))
    pr = problem([n], [1.0 / n], bc=[("prescribed", "transmissive")], states=(A.tolist(), B.tolist()),
                 lines={(0, 0): (-0.01, 0.0, 1.0)})
    dt = orc.cfl_dt(orc_params(orc, pr), W, 0.5)
    results = []
    for t0 in (0.01 - 0.75 * dt, 0.01 - 0.25 * dt, 0.01 + 0.25 * dt):
        Wg, Wsg, Wo, Wso, bad = compare_step(orc, pr, W, dt, t0)
        assert bad == 0
        assert_close(Wsg, Wso, what=f"W* t0={t0}")
        assert_close(Wg, Wo, what=f"t0={t0}")
        results.append(Wo)
    # B in both stages, B then A, A in both: three different steps
    assert np.abs(results[0] - results[1]).max() > 1e-8 and np.abs(results[1] - results[2]).max() > 1e-8
