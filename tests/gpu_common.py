"""Helpers of the GPU parity tests: run the same problem through the HIP
library (C ABI via paper_2309_10534_amd.tgks) and through the CPU oracle, each
from its own parameter structure built from one plain dict."""
import numpy as np

TOL_L1 = 1e-10  # L1-relative tolerance per component (GPU vs oracle, FP64)
# Per cell and component, on identical input: the device and the oracle
# differ by the rounding of their transcendental functions and fused
# products (a few ulps of each Gauss-point flux), which a step scales by
# dt / dx < 1; 1e-12 of the cell's own magnitude leaves three orders of
# magnitude for the sums of a step and no room for one wrong cell.
TOL_CELL = 1e-12


def problem(shape, dx, bc="transmissive", tau="inviscid", mu=0.0, prandtl=1.0, **kw):
    d = dict(shape=list(shape), dx=list(dx), bc=bc, tau=tau, mu=mu, prandtl=prandtl)
    d.update(kw)
    return d


def gpu_params(pr):
    from paper_2309_10534_amd import tgks
    kw = {k: v for k, v in pr.items() if k not in ("shape", "dx", "bc")}
    return tgks.tgks_params_default(len(pr["shape"]), pr["shape"], pr["dx"], pr["bc"], **kw)


def orc_params(orc, pr):
    kw = {k: v for k, v in pr.items() if k not in ("shape", "dx", "bc")}
    return orc.make_params(pr["shape"], pr["dx"], bc=pr["bc"], **kw)


class GpuProblem:
    """A context plus device buffers for one grid."""

    def __init__(self, pr):
        import torch
        from paper_2309_10534_amd import tgks
        self.t = tgks
        self.torch = torch
        self.pr = pr
        self.ctx = tgks.tgks_create(gpu_params(pr))
        self.n = tgks.tgks_state_size(self.ctx)

    def close(self):
        if self.ctx:
            self.t.tgks_destroy(self.ctx)
            self.ctx = None

    def dev(self, W):
        return self.torch.from_numpy(np.ascontiguousarray(W, dtype=np.float64)).cuda()

    def step(self, W, dt, flags=True, t0=None):
        torch = self.torch
        if t0 is not None:
            self.t.tgks_set_time(self.ctx, t0)
        Win = self.dev(W)
        Wout = torch.empty_like(Win)
        Ws = torch.empty_like(Win)
        dtd = torch.tensor([dt], dtype=torch.float64, device="cuda")
        fl = torch.zeros(self.t.tgks_flag_bytes(self.ctx), dtype=torch.uint8, device="cuda") if flags else None
        self.t.tgks_reset_status(self.ctx)
        self.t.tgks_step(self.ctx, Win, Wout, dtd, fl, Ws)
        bad = self.t.tgks_status(self.ctx)
        self.fallbacks = self.t.tgks_fallback_count(self.ctx)
        torch.cuda.synchronize()
        return (Wout.cpu().numpy().reshape(W.shape), Ws.cpu().numpy().reshape(W.shape),
                fl.cpu().numpy() if flags else None, bad)

    def cfl_dt(self, W, cfl, t=0.0, t_end=0.0):
        torch = self.torch
        dtd = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.t.tgks_cfl_dt(self.ctx, self.dev(W), cfl, t, t_end, dtd)
        return float(dtd.cpu()[0])

    def run(self, W, n_steps, cfl=0.0, t_end=0.0, fixed_dt=0.0, use_graph=False, t0=None):
        torch = self.torch
        if t0 is not None:
            self.t.tgks_set_time(self.ctx, t0)
        Wd = self.dev(W)
        td = torch.zeros(2, dtype=torch.float64, device="cuda")
        self.t.tgks_reset_status(self.ctx)
        self.t.tgks_run(self.ctx, Wd, n_steps, cfl, t_end, fixed_dt, td, use_graph)
        bad = self.t.tgks_status(self.ctx)
        torch.cuda.synchronize()
        return Wd.cpu().numpy().reshape(W.shape), td.cpu().numpy(), bad


def l1rel(a, b):
    """Per-component L1-relative difference sum|a-b| / sum|b|."""
    nc = a.shape[0]
    a2, b2 = a.reshape(nc, -1), b.reshape(nc, -1)
    return np.abs(a2 - b2).sum(axis=1) / np.maximum(np.abs(b2).sum(axis=1), 1e-300)


def cell_scale(b):
    """Magnitude of each cell's components: |b|, momenta at least
    sqrt(rho E) (a momentum that vanishes, as across a uniform direction or
    at rest, has no scale of its own)."""
    D = b.shape[0] - 2
    s = np.abs(b)
    ref = np.sqrt(np.abs(b[0] * b[D + 1]))
    for c in range(1, D + 1):
        s[c] = np.maximum(s[c], ref)
    return np.maximum(s, 1e-300)


def assert_cells(a, b, tol=TOL_CELL, what=""):
    """Element-wise bound: every component of every cell within tol of its
    own magnitude."""
    assert np.all(np.isfinite(a)), f"{what}: non-finite GPU values"
    e = np.abs(a - b) / cell_scale(b)
    k = int(np.argmax(e))
    worst = float(e.reshape(-1)[k])
    assert worst <= tol, f"{what}: cell difference {worst:.3e} > {tol} at {np.unravel_index(k, e.shape)}"
    return worst


def assert_close(a, b, tol=TOL_L1, what="", cell_tol=None):
    """L1-relative bound per component and, for parity on identical input
    (tol <= 1e-10), the element-wise bound of assert_cells."""
    e = l1rel(a, b)
    assert np.all(np.isfinite(a)), f"{what}: non-finite GPU values"
    assert np.all(e <= tol), f"{what}: L1-relative difference {e} > {tol}"
    if cell_tol is None and tol <= TOL_L1:
        cell_tol = TOL_CELL
    if cell_tol is not None:
        assert_cells(a, b, cell_tol, what)
    return e


def close_scaled(a, b, tol, what):
    """L1 difference per component relative to its L1 norm, momenta against
    the density's norm (a momentum that is zero up to rounding, as across a
    uniform direction, has no scale of its own)."""
    D = a.shape[0] - 2
    assert np.all(np.isfinite(a)), f"{what}: non-finite GPU values"
    for c in range(D + 2):
        scale = np.abs(b[c]).sum()
        if 1 <= c <= D:
            scale = max(scale, np.abs(b[0]).sum())
        e = np.abs(a[c] - b[c]).sum() / scale
        assert e <= tol, f"{what}: component {c} L1 difference {e} > {tol}"
    if tol <= TOL_L1:
        assert_cells(a, b, TOL_CELL, what)
