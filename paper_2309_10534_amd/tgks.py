"""Python binding of the C ABI in include/tgks.h (argument marshalling only).

Every function has the name of the C entry point it calls.  Arrays are torch
tensors on the HIP device (float64, contiguous, layout [nc][nz][ny][x]); torch
supplies device memory and the current stream, every step of the method runs
in the library's HIP kernels.  A missing library raises; there is no
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libtgks.so")

BC_PERIODIC, BC_TRANSMISSIVE, BC_REFLECTIVE, BC_NOSLIP, BC_PRESCRIBED = 0, 1, 2, 3, 4
SCHEME_TENO_D, SCHEME_WENO_AO, SCHEME_TENO5, SCHEME_WENO_Z = 0, 1, 2, 3
_SCHEME = {"teno_d": 0, "weno_ao": 1, "teno5": 2, "weno_z": 3}
TAU_INVISCID, TAU_VISCOUS, TAU_ZERO = 0, 1, 2
_BC = {"periodic": 0, "transmissive": 1, "reflective": 2, "noslip": 3, "prescribed": 4}
_FAR = {"transmissive": 1, "reflective": 2, "state_b": 4}
_TAU = {"inviscid": 0, "viscous": 1, "zero": 2}

KERNEL_KINDS = {"face_x": 0, "face_y": 1, "face_z": 2, "recon3d": 3, "update1": 4, "update2": 5, "cfl": 6}


class TgksParams(C.Structure):
    """Mirror of struct tgks_params."""
    _fields_ = [
        ("ndim", C.c_int32), ("n", C.c_int32 * 3), ("dx", C.c_double * 3),
        ("bc_lo", C.c_int32 * 3), ("bc_hi", C.c_int32 * 3),
        ("gamma", C.c_double), ("mu", C.c_double), ("prandtl", C.c_double),
        ("tau_mode", C.c_int32), ("c1", C.c_double), ("c2", C.c_double),
        ("ct1", C.c_double), ("ct2", C.c_double), ("ct1_tan", C.c_double), ("ct2_tan", C.c_double),
        ("eps", C.c_double), ("q", C.c_int32), ("recon", C.c_int32),
        ("bc_state", (C.c_double * 5) * 2), ("bc_line", ((C.c_double * 3) * 2) * 3),
        ("bc_far", (C.c_int32 * 2) * 3), ("fallback", C.c_int32),
        ("scheme", C.c_int32), ("d_hi", C.c_double), ("d_lo", C.c_double), ("eps_w", C.c_double),
    ]


class TgksError(RuntimeError):
    pass


_lib = None


def lib():
    """Open libtgks.so (built by ``python -m paper_2309_10534_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise TgksError(f"{LIB_PATH} not found: build it with `python -m paper_2309_10534_amd.build`")
    L = C.CDLL(LIB_PATH)
    P = C.POINTER(TgksParams)
    vp = C.c_void_p
    L.tgks_params_default.argtypes = [P, C.c_int32]
    L.tgks_create.argtypes = [P, vp, C.POINTER(vp)]
    L.tgks_destroy.argtypes = [vp]
    L.tgks_set_stream.argtypes = [vp, vp]
    L.tgks_state_size.argtypes = [vp]
    L.tgks_state_size.restype = C.c_int64
    L.tgks_flag_bytes.argtypes = [vp]
    L.tgks_flag_bytes.restype = C.c_int64
    L.tgks_cfl_dt.argtypes = [vp, vp, C.c_double, C.c_double, C.c_double, vp]
    L.tgks_step.argtypes = [vp, vp, vp, vp, vp, vp]
    L.tgks_run.argtypes = [vp, vp, C.c_int32, C.c_double, C.c_double, C.c_double, vp, C.c_int32]
    L.tgks_set_time.argtypes = [vp, C.c_double]
    L.tgks_fallback_count.argtypes = [vp, C.POINTER(C.c_int64)]
    L.tgks_status.argtypes = [vp, C.POINTER(C.c_int64)]
    L.tgks_reset_status.argtypes = [vp]
    L.tgks_timing.argtypes = [vp, C.c_int32]
    L.tgks_kernel_time.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    L.tgks_flop_counts.argtypes = [P, C.POINTER(C.c_double), C.c_int32]
    L.tgks_set_tile.argtypes = [vp, C.c_int32]
    L.tgks_tune.argtypes = [vp, vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_float)]
    dp = C.POINTER(C.c_double)
    L.tgks_measure_peaks.argtypes = [vp, dp, dp]
    L.tgks_measure_peaks.restype = C.c_int
    L.tgks_gp_flux_host.argtypes = [P, dp, dp, dp, dp, C.c_double, dp]
    L.tgks_teno_flag_host.argtypes = [P, dp, C.c_int32]
    L.tgks_teno_flag_host.restype = C.c_int
    L.tgks_erfc_host.argtypes = [C.c_double]
    L.tgks_erfc_host.restype = C.c_double
    L.tgks_step_adjoint.argtypes = [vp, vp, vp, vp, vp, vp]
    L.tgks_step_adjoint.restype = C.c_int
    L.tgks_gp_flux_vjp_host.argtypes = [P, dp, dp, dp, dp, C.c_double, dp, dp]
    L.tgks_gp_flux_vjp_host.restype = C.c_int
    bp = C.POINTER(C.c_int64)
    L.tgks_noalloc_capacity.argtypes = []
    L.tgks_noalloc_capacity.restype = C.c_int64
    L.tgks_noalloc_need.argtypes = [P]
    L.tgks_noalloc_need.restype = C.c_int64
    L.tgks_step_noalloc.argtypes = [P, vp, vp, vp, vp, vp, vp, bp]
    L.tgks_step_noalloc.restype = C.c_int
    L.tgks_batch_create.argtypes = [P, C.c_int32, vp, C.POINTER(vp)]
    L.tgks_batch_destroy.argtypes = [vp]
    L.tgks_batch_set_stream.argtypes = [vp, vp]
    L.tgks_batch_state_size.argtypes = [vp]
    L.tgks_batch_state_size.restype = C.c_int64
    L.tgks_batch_offsets.argtypes = [vp, bp]
    L.tgks_batch_run.argtypes = [vp, vp, C.c_int32, C.c_double, C.c_double, vp, C.c_int32]
    L.tgks_batch_status.argtypes = [vp, bp]
    L.tgks_batch_steps.argtypes = [vp, bp]
    L.tgks_batch_reset_status.argtypes = [vp]
    L.tgks_batch_set_tile.argtypes = [vp, C.c_int32]
    L.tgks_batch_tune.argtypes = [vp, vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_float)]
    for f in ("tgks_batch_create", "tgks_batch_destroy", "tgks_batch_set_stream", "tgks_batch_offsets",
              "tgks_batch_run", "tgks_batch_status", "tgks_batch_steps", "tgks_batch_reset_status",
              "tgks_batch_set_tile", "tgks_batch_tune"):
        getattr(L, f).restype = C.c_int
    for f in ("tgks_params_default", "tgks_create", "tgks_destroy", "tgks_set_stream", "tgks_cfl_dt", "tgks_step",
              "tgks_run", "tgks_status", "tgks_reset_status", "tgks_timing", "tgks_kernel_time",
              "tgks_flop_counts", "tgks_gp_flux_host", "tgks_set_tile", "tgks_tune", "tgks_set_time",
              "tgks_fallback_count"):
        getattr(L, f).restype = C.c_int
    _lib = L
    return L


def _check(rc, what):
    if rc != 0:
        raise TgksError(f"{what} returned {rc}" + (" (invalid argument)" if rc == -1 else " (HIP error)"))


def _ptr(t, numel=None, dtype=None):
    """Device pointer of a contiguous float64 (or uint8) HIP tensor, or None."""
    if t is None:
        return None
    import torch
    if not t.is_cuda:
        raise TgksError("expected a tensor on the HIP device")
    if not t.is_contiguous():
        raise TgksError("expected a contiguous tensor")
    if t.dtype != (dtype or torch.float64):
        raise TgksError(f"expected dtype {dtype or torch.float64}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise TgksError(f"expected {numel} elements, got {t.numel()}")
    return t.data_ptr()


def tgks_params_default(ndim, shape=None, dx=None, bc="transmissive", **kw):
    """tgks_params filled with the paper's constants; shape / dx / bc / keyword
    fields (gamma, mu, prandtl, tau, c1, c2, ct1, ct2, ct1_tan, ct2_tan, eps, q,
    recon: 0 conservative, 1 characteristic variables, fallback: 1 first-order
    fallback at non-physical Gauss-point states, scheme: "teno_d" (default),
    "weno_ao", "teno5" (q 6 unless given) or "weno_z", d_hi, d_lo, eps_w)
    override them.  Prescribed
    sides (bc name "prescribed"): states = (A, B), lines = {(axis, end):
    (s0, s_n, s_t)}, far = {(axis, end): "transmissive" | "reflective" |
    "state_b"} (see tgks.h)."""
    p = TgksParams()
    _check(lib().tgks_params_default(C.byref(p), int(ndim)), "tgks_params_default")
    if shape is not None:
        for d in range(ndim):
            p.n[d] = int(shape[d])
    if dx is not None:
        for d in range(ndim):
            p.dx[d] = float(dx[d])
    for d in range(ndim):
        lo, hi = (bc, bc) if isinstance(bc, str) else bc[d]
        p.bc_lo[d], p.bc_hi[d] = _BC[lo], _BC[hi]
    if "tau" in kw:
        p.tau_mode = _TAU[kw.pop("tau")]
    if "scheme" in kw:
        sch = kw.pop("scheme")
        p.scheme = _SCHEME[sch] if isinstance(sch, str) else int(sch)
        if p.scheme == SCHEME_TENO5 and "q" not in kw:
            p.q = 6  # the TENO5 power of Sec. 4.1
    states, lines, far = kw.pop("states", None), kw.pop("lines", None), kw.pop("far", None)
    if states is not None:
        for k in range(2):
            for c, v in enumerate(states[k]):
                p.bc_state[k][c] = float(v)
    for (d, e), ln in (lines or {}).items():
        for k in range(3):
            p.bc_line[d][e][k] = float(ln[k])
    for d in range(3):
        for e in range(2):
            p.bc_far[d][e] = _FAR["state_b"]
    for (d, e), name in (far or {}).items():
        p.bc_far[d][e] = _FAR[name]
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def tgks_create(params, stream=None):
    """Context handle (int).  stream: torch.cuda.Stream or None for the current stream."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    h = C.c_void_p()
    _check(lib().tgks_create(C.byref(params), C.c_void_p(s.cuda_stream), C.byref(h)), "tgks_create")
    return h.value


def tgks_destroy(ctx):
    _check(lib().tgks_destroy(ctx), "tgks_destroy")


def tgks_set_stream(ctx, stream):
    _check(lib().tgks_set_stream(ctx, C.c_void_p(stream.cuda_stream)), "tgks_set_stream")


def tgks_state_size(ctx):
    return int(lib().tgks_state_size(ctx))


def tgks_flag_bytes(ctx):
    return int(lib().tgks_flag_bytes(ctx))


def tgks_cfl_dt(ctx, W, cfl, t, t_end, dt_dev):
    n = tgks_state_size(ctx)
    _check(lib().tgks_cfl_dt(ctx, _ptr(W, n), float(cfl), float(t), float(t_end), _ptr(dt_dev, 1)), "tgks_cfl_dt")


def tgks_step(ctx, W_in, W_out, dt_dev, flags=None, W_star=None):
    import torch
    n = tgks_state_size(ctx)
    fl = _ptr(flags, tgks_flag_bytes(ctx), torch.uint8) if flags is not None else None
    _check(lib().tgks_step(ctx, _ptr(W_in, n), _ptr(W_out, n), _ptr(dt_dev, 1), fl, _ptr(W_star, n)), "tgks_step")


def tgks_noalloc_capacity():
    """Doubles of the scratch array of tgks_step_noalloc."""
    return int(lib().tgks_noalloc_capacity())


def tgks_noalloc_need(params):
    """Doubles of scratch one tgks_step_noalloc of this grid uses."""
    return int(lib().tgks_noalloc_need(C.byref(params)))


def tgks_step_noalloc(params, W_in, W_out, dt_dev, flags=None, W_star=None, stream=None, failures=False):
    """tgks_step without a context: the library allocates nothing (its work
    buffers are a fixed device array).  failures=True synchronises and
    returns the count of non-physical Gauss-point evaluations."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    D, nc = params.ndim, params.ndim + 2
    cells = params.n[0] * params.n[1] * params.n[2]
    n = nc * cells
    fl = None
    if flags is not None:
        # flag buffer of include/tgks.h: normal planes, then the tangential ones
        faces = sum(cells // params.n[d] * (params.n[d] + 1) for d in range(D))
        fl = _ptr(flags, D * n + (4 if D == 2 else 16 if D == 3 else 0) * nc * faces, torch.uint8)
    f = C.c_int64(0)
    _check(lib().tgks_step_noalloc(C.byref(params), C.c_void_p(s.cuda_stream), _ptr(W_in, n), _ptr(W_out, n),
                                   _ptr(dt_dev, 1), fl, _ptr(W_star, n), C.byref(f) if failures else None),
           "tgks_step_noalloc")
    return f.value if failures else None


def tgks_run(ctx, W, n_steps, cfl=0.0, t_end=0.0, fixed_dt=0.0, time_dev=None, use_graph=False):
    n = tgks_state_size(ctx)
    _check(lib().tgks_run(ctx, _ptr(W, n), int(n_steps), float(cfl), float(t_end), float(fixed_dt),
                          _ptr(time_dev, 2), int(bool(use_graph))), "tgks_run")


def tgks_set_time(ctx, t0):
    """Time of the state that the next tgks_step / tgks_run advances (the
    prescribed boundary states depend on it)."""
    _check(lib().tgks_set_time(ctx, float(t0)), "tgks_set_time")


def tgks_fallback_count(ctx):
    """Gauss-point side states replaced by the first-order fallback since
    the last reset (synchronises)."""
    v = C.c_int64()
    _check(lib().tgks_fallback_count(ctx, C.byref(v)), "tgks_fallback_count")
    return v.value


def tgks_status(ctx):
    v = C.c_int64()
    _check(lib().tgks_status(ctx, C.byref(v)), "tgks_status")
    return v.value


def tgks_reset_status(ctx):
    _check(lib().tgks_reset_status(ctx), "tgks_reset_status")


def tgks_timing(ctx, enable):
    _check(lib().tgks_timing(ctx, int(bool(enable))), "tgks_timing")


def tgks_kernel_time(ctx, kind):
    """(milliseconds, launches) summed over the launches of one kernel kind."""
    ms = C.c_double()
    n = C.c_int64()
    k = KERNEL_KINDS[kind] if isinstance(kind, str) else int(kind)
    _check(lib().tgks_kernel_time(ctx, k, C.byref(ms), C.byref(n)), "tgks_kernel_time")
    return ms.value, n.value


def tgks_flop_counts(params):
    """Algorithmic operation counts (see include/tgks.h) as a dict."""
    out = (C.c_double * 8)()
    _check(lib().tgks_flop_counts(C.byref(params), out, 8), "tgks_flop_counts")
    keys = ("normal", "face", "face_stage2", "update1", "update2", "face_transcendentals", "face_divisions", "cfl")
    return {k: out[i] for i, k in enumerate(keys)}


def tgks_teno_flag_host(params, Q, fast=1):
    """The kernels' TENO-D selection of five host values (verification).
    fast: 0 exact weights, 1 the 3-D kernels' evaluation, 2 the 1-D/2-D
    kernels' (a bool selects 0 or 1)."""
    q = (C.c_double * 5)(*[float(v) for v in Q])
    f = lib().tgks_teno_flag_host(C.byref(params), q, int(fast))
    if f < 0:
        raise TgksError("tgks_teno_flag_host: invalid argument")
    return f


def tgks_erfc_host(x):
    """The kernels' erfc (half-space moments) evaluated on the host."""
    return lib().tgks_erfc_host(float(x))


def tgks_measure_peaks(stream=None):
    """(FP64 FMA TFLOP/s, copy GB/s) measured on the current device."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    t, b = C.c_double(), C.c_double()
    _check(lib().tgks_measure_peaks(C.c_void_p(s.cuda_stream), C.byref(t), C.byref(b)), "tgks_measure_peaks")
    return t.value, b.value


def tgks_gp_flux_host(params, Wl, Wr, dWl, dWr, dt):
    """Host evaluation of the device Gauss-point flux (numpy in, numpy out):
    returns (F[2][nc] for dt and dt/2, ok)."""
    import numpy as np
    D = params.ndim
    nc = D + 2

    def buf(x, n):
        a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
        assert a.size == n
        return a

    l, r = buf(Wl, nc), buf(Wr, nc)
    dl, dr = buf(dWl, D * nc), buf(dWr, D * nc)
    F = np.zeros(2 * nc)
    P = C.POINTER(C.c_double)
    rc = lib().tgks_gp_flux_host(C.byref(params), l.ctypes.data_as(P), r.ctypes.data_as(P), dl.ctypes.data_as(P),
                                 dr.ctypes.data_as(P), float(dt), F.ctypes.data_as(P))
    if rc < 0:
        raise TgksError("tgks_gp_flux_host: invalid argument")
    return F.reshape(2, nc), rc == 0


def tgks_set_tile(ctx, tile):
    _check(lib().tgks_set_tile(ctx, int(tile)), "tgks_set_tile")


def tgks_tune(ctx, W, steps=3):
    """Time every 2-D tile shape on the state W, keep the fastest; returns
    (chosen index, [ms per step of each shape])."""
    n = tgks_state_size(ctx)
    ch = C.c_int32()
    ms = (C.c_float * 3)()
    _check(lib().tgks_tune(ctx, _ptr(W, n), int(steps), C.byref(ch), ms), "tgks_tune")
    return ch.value, [ms[i] for i in range(3)]


# ---------------------------------------------------------------------------
# batched runs
# ---------------------------------------------------------------------------
class _Batch:
    """Handle of a tgks_batch with its instance count."""

    def __init__(self, handle, n_inst):
        self.handle = handle
        self.n_inst = n_inst


def tgks_batch_create(params_list, stream=None):
    """Batch of len(params_list) grids (TgksParams each, same ndim)."""
    import torch
    n = len(params_list)
    arr = (TgksParams * n)(*params_list)
    s = stream if stream is not None else torch.cuda.current_stream()
    h = C.c_void_p()
    _check(lib().tgks_batch_create(arr, n, C.c_void_p(s.cuda_stream), C.byref(h)), "tgks_batch_create")
    return _Batch(h.value, n)


def tgks_batch_destroy(b):
    _check(lib().tgks_batch_destroy(b.handle), "tgks_batch_destroy")


def tgks_batch_set_stream(b, stream):
    _check(lib().tgks_batch_set_stream(b.handle, C.c_void_p(stream.cuda_stream)), "tgks_batch_set_stream")


def tgks_batch_state_size(b):
    return int(lib().tgks_batch_state_size(b.handle))


def tgks_batch_offsets(b):
    """State offsets (doubles) of the instances in a packed state, n_inst + 1 entries."""
    out = (C.c_int64 * (b.n_inst + 1))()
    _check(lib().tgks_batch_offsets(b.handle, out), "tgks_batch_offsets")
    return [int(x) for x in out]


def tgks_batch_run(b, W, n_steps, cfl, t_end=0.0, time_dev=None, use_graph=False):
    n = tgks_batch_state_size(b)
    _check(lib().tgks_batch_run(b.handle, _ptr(W, n), int(n_steps), float(cfl), float(t_end),
                                _ptr(time_dev, 2 * b.n_inst), int(bool(use_graph))), "tgks_batch_run")


def tgks_batch_status(b):
    out = (C.c_int64 * b.n_inst)()
    _check(lib().tgks_batch_status(b.handle, out), "tgks_batch_status")
    return [int(x) for x in out]


def tgks_batch_steps(b):
    """Steps each instance took in the last run."""
    out = (C.c_int64 * b.n_inst)()
    _check(lib().tgks_batch_steps(b.handle, out), "tgks_batch_steps")
    return [int(x) for x in out]


def tgks_batch_reset_status(b):
    _check(lib().tgks_batch_reset_status(b.handle), "tgks_batch_reset_status")


def tgks_batch_set_tile(b, tile):
    _check(lib().tgks_batch_set_tile(b.handle, int(tile)), "tgks_batch_set_tile")


def tgks_batch_tune(b, W, steps=2):
    """Time every 2-D tile shape on the packed state W, keep the fastest;
    returns (chosen index, [ms per batched step of each shape])."""
    n = tgks_batch_state_size(b)
    ch = C.c_int32()
    ms = (C.c_float * 3)()
    _check(lib().tgks_batch_tune(b.handle, _ptr(W, n), int(steps), C.byref(ch), ms), "tgks_batch_tune")
    return ch.value, [ms[i] for i in range(3)]


def pack(states):
    """Concatenate instance states (numpy arrays) into one packed host array."""
    import numpy as np
    return np.concatenate([np.ascontiguousarray(s, dtype=np.float64).reshape(-1) for s in states])


def unpack(packed, offsets, shapes):
    """Views of the instances' states in a packed array (numpy or torch)."""
    return [packed[offsets[i]:offsets[i + 1]].reshape(shapes[i]) for i in range(len(shapes))]


# ---------------------------------------------------------------------------
# reverse mode
# ---------------------------------------------------------------------------
def tgks_step_adjoint(ctx, W_n, dt_dev, gW_out, gW_in, W_star=None):
    """gW_in = (dW_out/dW_in)^T gW_out for one step from W_n (dt and the stencil
    selections frozen).  W_star: the step's W* from tgks_step, or None."""
    n = tgks_state_size(ctx)
    _check(lib().tgks_step_adjoint(ctx, _ptr(W_n, n), _ptr(W_star, n), _ptr(dt_dev, 1), _ptr(gW_out, n),
                                   _ptr(gW_in, n)), "tgks_step_adjoint")


def tgks_gp_flux_vjp_host(params, Wl, Wr, dWl, dWr, dt, Fb):
    """Host reverse of the Gauss-point flux: Fb (2, nc) -> (Wl_b, Wr_b, dWl_b, dWr_b)."""
    import numpy as np
    D = params.ndim
    nc = D + 2

    def buf(x, n):
        a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
        assert a.size == n
        return a

    P = C.POINTER(C.c_double)
    args = [buf(Wl, nc), buf(Wr, nc), buf(dWl, D * nc), buf(dWr, D * nc)]
    fb = buf(Fb, 2 * nc)
    G = np.zeros(2 * nc + 2 * D * nc)
    rc = lib().tgks_gp_flux_vjp_host(C.byref(params), *[a.ctypes.data_as(P) for a in args], float(dt),
                                     fb.ctypes.data_as(P), G.ctypes.data_as(P))
    if rc < 0:
        raise TgksError("tgks_gp_flux_vjp_host: invalid argument")
    return G[:nc], G[nc:2 * nc], G[2 * nc:2 * nc + D * nc].reshape(D, nc), G[2 * nc + D * nc:].reshape(D, nc)
