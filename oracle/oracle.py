"""ctypes wrapper of the CPU FP64 oracle (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use this module.  It loads ``liboracle.so`` built from
``gks_oracle.cpp`` by ``oracle/build.py`` and shares nothing with the HIP path.

Arrays follow the layout [component][z][y][x] (x fastest), components
(rho, rho U, rho V, rho W, rho E) truncated to D+2.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

BC = {"periodic": 0, "transmissive": 1, "reflective": 2, "noslip": 3, "prescribed": 4}
FAR = {"transmissive": 1, "reflective": 2, "state_b": 4}
TAU = {"inviscid": 0, "viscous": 1, "zero": 2}


class OrcParams(C.Structure):
    _fields_ = [
        ("ndim", C.c_int), ("n", C.c_int * 3), ("dx", C.c_double * 3),
        ("bc_lo", C.c_int * 3), ("bc_hi", C.c_int * 3),
        ("gamma", C.c_double), ("mu", C.c_double), ("prandtl", C.c_double),
        ("tau_mode", C.c_int), ("c1", C.c_double), ("c2", C.c_double),
        ("ct1", C.c_double), ("ct2", C.c_double), ("ct1_tan", C.c_double), ("ct2_tan", C.c_double),
        ("eps", C.c_double), ("q", C.c_int), ("recon", C.c_int),
        ("bc_state", (C.c_double * 5) * 2), ("bc_line", ((C.c_double * 3) * 2) * 3),
        ("bc_far", (C.c_int * 2) * 3), ("fallback", C.c_int),
        ("scheme", C.c_int), ("d_hi", C.c_double), ("d_lo", C.c_double), ("eps_w", C.c_double),
    ]


SCHEME = {"teno_d": 0, "weno_ao": 1, "teno5": 2, "weno_z": 3}


_lib = None


def use_library(path):
    """Load the oracle from another build of gks_oracle.cpp (the CPU
    baseline's -march=native build); must precede the first call."""
    global LIB_PATH, _lib
    if _lib is not None:
        raise RuntimeError("the oracle library is already loaded")
    LIB_PATH = path


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        u8 = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
        P = C.POINTER(OrcParams)
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_beta.argtypes = [dp, dp]
        L.orc_teno_select.argtypes = [dp, C.c_double, C.c_double, C.c_double, C.c_int]
        L.orc_teno_face.argtypes = [dp, C.c_double, C.c_double, C.c_double, C.c_int, dp]
        L.orc_teno_gauss.argtypes = [dp, C.c_double, C.c_double, C.c_double, C.c_int, dp]
        L.orc_teno_eval.argtypes = [dp, C.c_int, C.c_int, dp]
        L.orc_recon.argtypes = [P, dp, C.c_int, dp]
        L.orc_teno_gauss_canonical.argtypes = [dp, C.c_int, dp]
        L.orc_lin_weights.argtypes = [C.c_int, dp]
        L.orc_moments.argtypes = [C.c_double, C.c_double, C.c_int, dp]
        L.orc_micro_slope.argtypes = [C.c_int, C.c_double, dp, dp, dp]
        L.orc_moment_mono.argtypes = [C.c_int, C.c_double, dp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]
        L.orc_moment_mono.restype = C.c_double
        L.orc_gp_flux.argtypes = [P, dp, dp, dp, dp, C.c_double, C.c_int, dp, dp, dp, dp]
        L.orc_gp_flux_dual.argtypes = [P, dp, dp, dp, dp, dp, dp, dp, dp, C.c_double, C.c_int, dp, dp, dp]
        L.orc_char_basis.argtypes = [C.c_int, C.c_double, dp, C.c_int, dp, dp]
        L.orc_char_recon.argtypes = [P, dp, C.c_double, dp, C.c_void_p]
        L.orc_flag_bytes.argtypes = [P]
        L.orc_flag_bytes.restype = C.c_long
        L.orc_step.argtypes = [P, dp, dp, C.c_double, C.c_void_p, C.c_void_p, C.c_double, C.POINTER(C.c_long)]
        L.orc_step.restype = C.c_long
        L.orc_step_dual.argtypes = [P, dp, dp, dp, dp, C.c_double]
        L.orc_step_dual.restype = C.c_long
        L.orc_cfl_dt.argtypes = [P, dp, C.c_double, C.POINTER(C.c_double)]
        L.orc_run.argtypes = [P, dp, C.c_int, C.c_double, C.c_double, C.c_double,
                              C.POINTER(C.c_double), C.POINTER(C.c_int), C.c_double]
        L.orc_run.restype = C.c_long
        _ = u8
        _lib = L
    return _lib


def set_threads(n: int) -> int:
    return lib().orc_set_threads(int(n))


def make_params(shape, dx, bc="transmissive", gamma=1.4, mu=0.0, prandtl=1.0, tau="inviscid",
                c1=0.01, c2=1.0, ct1=1e-7, ct2=1e-5, ct1_tan=None, ct2_tan=None, eps=1e-40, q=None,
                recon=0, states=None, lines=None, far=None, fallback=0, scheme="teno_d", d_hi=0.85,
                d_lo=0.85, eps_w=1e-8):
    """shape: cells per axis (x, y, z) truncated to D; bc: one name or a list of
    (lo, hi) names per axis; recon: 0 conservative, 1 characteristic variables
    (1-D, 2-D).  Prescribed sides ("prescribed", 1-D and 2-D): states = (A, B)
    conservative states; lines = {(axis, end): (s0, s_n, s_t)}; far =
    {(axis, end): "transmissive" | "reflective" | "state_b"}: the ghost cell
    centred at (s, r) holds A where s < (s0 + s_n r) + s_t t, else what far
    gives.  fallback = 1: first-order fallback at non-physical Gauss-point
    states (1-D, 2-D; not in the paper).  scheme: "teno_d" (Sec. 4.2, the
    default), or one of the paper's comparison schemes on 1-D and 2-D grids
    with conservative variables: "weno_ao" (Sec. 3.2; linear weights d_hi,
    d_lo, epsilon eps_w), "teno5" (Sec. 4.1; C_T = ct1, epsilon eps, q = 6
    unless given), "weno_z" (Sec. 3.1; epsilon eps_w)."""
    p = OrcParams()
    D = len(shape)
    p.ndim = D
    for d in range(3):
        p.n[d] = int(shape[d]) if d < D else 1
        p.dx[d] = float(dx[d]) if d < D else 1.0
        if isinstance(bc, str):
            lo = hi = bc
        else:
            lo, hi = bc[d] if d < D else ("transmissive", "transmissive")
        p.bc_lo[d] = BC[lo]
        p.bc_hi[d] = BC[hi]
    p.gamma, p.mu, p.prandtl = gamma, mu, prandtl
    p.tau_mode = TAU[tau]
    p.c1, p.c2 = c1, c2
    p.ct1, p.ct2 = ct1, ct2
    p.ct1_tan = ct1 if ct1_tan is None else ct1_tan
    p.ct2_tan = ct2 if ct2_tan is None else ct2_tan
    p.scheme = SCHEME[scheme] if isinstance(scheme, str) else int(scheme)
    # q: 7 for TENO-D (Sec. 4.2), 6 for TENO5 (Sec. 4.1)
    p.eps, p.q = eps, (6 if p.scheme == 2 else 7) if q is None else q
    p.d_hi, p.d_lo, p.eps_w = d_hi, d_lo, eps_w
    p.recon = int(recon)
    p.fallback = int(fallback)
    if states is not None:
        for k in range(2):
            for c, v in enumerate(states[k]):
                p.bc_state[k][c] = float(v)
    for (d, e), ln in (lines or {}).items():
        for k in range(3):
            p.bc_line[d][e][k] = float(ln[k])
    for d in range(3):
        for e in range(2):
            p.bc_far[d][e] = FAR["state_b"]
    for (d, e), name in (far or {}).items():
        p.bc_far[d][e] = FAR[name]
    return p


def _arr(W):
    return np.ascontiguousarray(W, dtype=np.float64)


def teno_face(Q, ct1=1e-7, ct2=1e-5, eps=1e-40, q=7):
    out = np.zeros(4)
    f = lib().orc_teno_face(_arr(Q), ct1, ct2, eps, q, out)
    return out, f


def teno_gauss(Q, ct1=1e-7, ct2=1e-5, eps=1e-40, q=7):
    out = np.zeros(4)
    f = lib().orc_teno_gauss(_arr(Q), ct1, ct2, eps, q, out)
    return out, f


def teno_eval(Q, flag, gauss=False):
    out = np.zeros(4)
    lib().orc_teno_eval(_arr(Q), int(flag), int(bool(gauss)), out)
    return out


def recon(params, Q, gauss=False):
    """Reconstruction of params' scheme from five values: (out, flags) with
    out = {v(-1/2), s(-1/2), v(+1/2), s(+1/2)} or, gauss=True, the values and
    derivatives at the Gauss points -+1/(2 sqrt 3) (cell units)."""
    out = np.zeros(4)
    f = lib().orc_recon(C.byref(params), _arr(Q), int(bool(gauss)), out)
    if f < 0:
        raise ValueError("invalid parameters")
    return out, f


def teno_gauss_canonical(Q, flag):
    """The 3-D first sweep's Gauss-point evaluation (canonical operation
    order) with a given flag: {v(s-), d(s-), v(s+), d(s+)}."""
    out = np.zeros(4)
    lib().orc_teno_gauss_canonical(_arr(Q), int(flag), out)
    return out


def lin_weights(where):
    """Linear weights of the three quadratics at x = -1/2, +1/2, s-, s+."""
    d = np.zeros(3)
    lib().orc_lin_weights(int(where), d)
    return d


def teno_select(Q, ct1=1e-7, ct2=1e-5, eps=1e-40, q=7):
    return lib().orc_teno_select(_arr(Q), ct1, ct2, eps, q)


def char_basis(D, gamma, Wb, a):
    """(L, R, ok): left eigenvectors (rows) and right eigenvectors (columns)
    of the Euler flux Jacobian along frame axis a at the frame-ordered state
    Wb; the identity and ok = False for a non-physical state."""
    nc = D + 2
    L, R = np.zeros((nc, nc)), np.zeros((nc, nc))
    ok = lib().orc_char_basis(int(D), float(gamma), _arr(Wb), int(a), L.reshape(-1), R.reshape(-1))
    if ok < 0:
        raise ValueError("bad arguments")
    return L, R, bool(ok)


def char_recon(P, cells, dx):
    """Characteristic normal reconstruction of one face from six frame-ordered
    cells (6 x nc): ({vl, sl, vr, sr} as a 4 x nc array, right-side flags)."""
    cells = _arr(cells)
    nc = cells.shape[1]
    out = np.zeros((4, nc))
    fr = np.zeros(5, dtype=np.uint8)
    lib().orc_char_recon(P, cells.reshape(-1), float(dx), out.reshape(-1), fr.ctypes.data)
    return out, fr[:nc]


def beta(Q):
    out = np.zeros(4)
    lib().orc_beta(_arr(Q), out)
    return out


def moments(U, lam, kind):
    out = np.zeros(10)
    lib().orc_moments(float(U), float(lam), int(kind), out)
    return out


def micro_slope(D, gamma, W, b):
    a = np.zeros(5)
    Wp = np.zeros(5)
    Wp[: D + 2] = W
    bp = np.zeros(5)
    bp[: D + 2] = b
    lib().orc_micro_slope(D, gamma, Wp, bp, a)
    return a[: D + 2]


def moment_mono(D, gamma, W, kind, e):
    Wp = np.zeros(5)
    Wp[: D + 2] = W
    return lib().orc_moment_mono(D, gamma, Wp, kind, *[int(x) for x in e])


def gp_flux(params, Wl, Wr, dWl, dWr, dt, deltas):
    """Flux at one Gauss point in the face frame.  dWl, dWr: (D, D+2)."""
    D = params.ndim
    nc = D + 2

    def pad(v):
        o = np.zeros(5)
        o[:nc] = v
        return o

    def padd(m):
        o = np.zeros((3, 5))
        m = np.asarray(m, dtype=np.float64)
        o[: m.shape[0], :nc] = m
        return o.ravel()

    deltas = np.asarray(deltas, dtype=np.float64)
    F = np.zeros((2, 5))
    W0 = np.zeros(5)
    dW0 = np.zeros((3, 5))
    bad = lib().orc_gp_flux(C.byref(params), pad(Wl), pad(Wr), padd(dWl), padd(dWr), float(dt),
                            len(deltas), deltas, F.ravel(), W0, dW0.ravel())
    if bad < 0:
        raise ValueError("invalid parameters")
    return F[: len(deltas), :nc].copy(), W0[:nc].copy(), dW0[:D, :nc].copy(), bad


def flag_bytes(params):
    return lib().orc_flag_bytes(C.byref(params))


def step(params, W, dt, want_flags=False, want_wstar=False, t=0.0, fallbacks=None):
    """One step of W, the state at time t (prescribed boundary states).
    fallbacks: a one-element list that receives the number of Gauss-point
    side states the first-order fallback replaced."""
    W = _arr(W)
    out = np.empty_like(W)
    flags = np.zeros(flag_bytes(params), dtype=np.uint8) if want_flags else None
    ws = np.empty_like(W) if want_wstar else None
    nfb = C.c_long(0)
    bad = lib().orc_step(C.byref(params), W, out, float(dt),
                         flags.ctypes.data if flags is not None else None,
                         ws.ctypes.data if ws is not None else None, float(t), C.byref(nfb))
    if bad < 0:
        raise ValueError("invalid parameters or dt")
    if fallbacks is not None:
        fallbacks[:] = [nfb.value]
    return out, flags, ws, bad


def step_dual(params, W, dW, dt):
    W = _arr(W)
    dW = _arr(dW)
    out = np.empty_like(W)
    dout = np.empty_like(W)
    bad = lib().orc_step_dual(C.byref(params), W, dW, out, dout, float(dt))
    if bad < 0:
        raise ValueError("invalid parameters or dt")
    return out, dout, bad


def gp_flux_dual(params, Wl, Wr, dWl, dWr, tWl, tWr, tdWl, tdWr, dt, deltas):
    """Flux at one Gauss point and its directional derivative along the
    tangent (tWl, tWr, tdWl, tdWr), dt constant.  Returns (F, dF), each
    (len(deltas), D+2)."""
    D = params.ndim
    nc = D + 2

    def pad(v):
        o = np.zeros(5)
        o[:nc] = v
        return o

    def padd(m):
        o = np.zeros((3, 5))
        m = np.asarray(m, dtype=np.float64)
        o[: m.shape[0], :nc] = m
        return o.ravel()

    deltas = np.asarray(deltas, dtype=np.float64)
    F = np.zeros((2, 5))
    dF = np.zeros((2, 5))
    bad = lib().orc_gp_flux_dual(C.byref(params), pad(Wl), pad(Wr), padd(dWl), padd(dWr), pad(tWl), pad(tWr),
                                 padd(tdWl), padd(tdWr), float(dt), len(deltas), deltas, F.ravel(), dF.ravel())
    if bad < 0:
        raise ValueError("invalid parameters")
    return F[: len(deltas), :nc].copy(), dF[: len(deltas), :nc].copy()


def cfl_dt(params, W, cfl):
    dt = C.c_double()
    if lib().orc_cfl_dt(C.byref(params), _arr(W), float(cfl), C.byref(dt)) != 0:
        raise ValueError("invalid parameters")
    return dt.value


def run(params, W, max_steps, cfl=0.5, t_end=0.0, fixed_dt=0.0, t0=0.0):
    """Advance a copy of W; returns (W, t, steps, failures).  t counts from 0;
    the prescribed boundary states are those of time t0 + t."""
    W = _arr(W).copy()
    t = C.c_double()
    s = C.c_int()
    bad = lib().orc_run(C.byref(params), W, int(max_steps), float(cfl), float(t_end),
                        float(fixed_dt), C.byref(t), C.byref(s), float(t0))
    if bad < 0:
        raise ValueError("invalid parameters or non-positive dt")
    return W, t.value, s.value, bad
