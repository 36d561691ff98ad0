"""Brute-force gas-kinetic interface flux by numerical quadrature.

An independent re-derivation of the oracle's Gauss-point flux, used only by the
tests.  Every moment is a numerical integral of the Maxwellian (Eq. 2.2) times
the integrand written out from the paper:
  * normal velocity u1: scipy.integrate.quad over u1 > 0 / u1 < 0 (half-space
    moments, Eq. 2.6) or Gauss-Hermite (full space);
  * tangential velocities: Gauss-Hermite nodes;
  * internal energy xi^2 (K Gaussian degrees of freedom, i.e. a Gamma(K/2)
    variable): generalised Gauss-Laguerre nodes;
  * micro coefficients: numpy.linalg.solve of <a psi> = b with the matrix of
    quadrature moments (Eq. 2.7);
  * time integrals of the factors of Eq. 2.5 over [0, delta]: scipy quad.
It shares no formula with the oracle's moment recursions, polynomial expansion
or Gaussian elimination.
"""
import math

import numpy as np
from scipy import integrate, special

NGH = 14
NGL = 10


class Gauss:
    """Maxwellian of a conservative state in the face frame (u1 normal)."""

    def __init__(self, W, D, gamma):
        self.D = D
        self.K = 2.0 / (gamma - 1.0) - D
        W = np.asarray(W, dtype=np.float64)
        self.rho = W[0]
        self.U = W[1:1 + D] / self.rho
        eint = W[D + 1] - 0.5 * self.rho * np.dot(self.U, self.U)
        self.p = (gamma - 1.0) * eint
        self.lam = self.rho / (2.0 * self.p)
        x, w = special.roots_hermite(NGH)
        self.gh_x, self.gh_w = x, w / math.sqrt(math.pi)
        a = self.K / 2.0 - 1.0
        xl, wl = special.roots_genlaguerre(NGL, a)
        self.gl_x = xl / self.lam
        self.gl_w = wl / special.gamma(self.K / 2.0)

    def expect(self, h, kind):
        """E[h(u1, u2, u3, xi2)] per unit density; kind 0 full, +1 u1>0, -1 u1<0."""
        lam = self.lam
        # tangential nodes (tensor grid) and xi^2 nodes
        tn = [self.U[d] + self.gh_x / math.sqrt(lam) for d in range(1, self.D)]
        tw = [self.gh_w for _ in range(1, self.D)]
        if self.D == 1:
            u2 = np.zeros(1); w2 = np.ones(1); u3 = np.zeros(1); w3 = np.ones(1)
        elif self.D == 2:
            u2, w2 = tn[0], tw[0]; u3 = np.zeros(1); w3 = np.ones(1)
        else:
            u2, w2, u3, w3 = tn[0], tw[0], tn[1], tw[1]
        U2, U3, X = np.meshgrid(u2, u3, self.gl_x, indexing="ij")
        Wt = np.einsum("i,j,k->ijk", w2, w3, self.gl_w)

        def inner(u1):
            return float(np.sum(Wt * h(u1, U2, U3, X)))

        U1, lam1 = self.U[0], lam

        def dens(u1):
            return math.sqrt(lam1 / math.pi) * math.exp(-lam1 * (u1 - U1) ** 2)

        if kind == 0:
            xs = U1 + self.gh_x / math.sqrt(lam)
            return float(sum(w * inner(x) for x, w in zip(xs, self.gh_w)))
        f = lambda u: dens(u) * inner(u)
        if kind > 0:
            v, _ = integrate.quad(f, 0.0, np.inf, epsabs=0.0, epsrel=1e-13, limit=200)
        else:
            v, _ = integrate.quad(f, -np.inf, 0.0, epsabs=0.0, epsrel=1e-13, limit=200)
        return v


def psi_list(D):
    """psi_alpha as functions of (u1, u2, u3, xi2)."""
    out = [lambda u1, u2, u3, x: 1.0 + 0.0 * u2]
    comps = [lambda u1, u2, u3, x: u1 + 0.0 * u2, lambda u1, u2, u3, x: u2 + 0.0 * u1,
             lambda u1, u2, u3, x: u3 + 0.0 * u1]
    out += comps[:D]

    def en(u1, u2, u3, x):
        s = u1 * u1 + x
        if D >= 2:
            s = s + u2 * u2
        if D >= 3:
            s = s + u3 * u3
        return 0.5 * s

    out.append(en)
    return out


def vel(d):
    return [lambda u1, u2, u3, x: u1, lambda u1, u2, u3, x: u2, lambda u1, u2, u3, x: u3][d]


def micro_fn(a, psis):
    return lambda u1, u2, u3, x: sum(a[b] * psis[b](u1, u2, u3, x) for b in range(len(a)))


def moment_matrix(g, psis):
    n = len(psis)
    M = np.zeros((n, n))
    for i in range(n):
        for j in range(i, n):
            M[i, j] = M[j, i] = g.expect(lambda *u, i=i, j=j: psis[i](*u) * psis[j](*u), 0)
    return M


def gp_flux_quadrature(D, gamma, Wl, Wr, dWl, dWr, dt, deltas, tau_mode="inviscid", c1=0.01, c2=1.0,
                       mu=0.0, prandtl=1.0):
    """Returns (F[len(deltas)][D+2], W0, dW0[D][D+2]) in the face frame."""
    psis = psi_list(D)
    nc = D + 2
    gl, gr = Gauss(Wl, D, gamma), Gauss(Wr, D, gamma)
    W0 = np.array([gl.rho * gl.expect(psis[a], +1) + gr.rho * gr.expect(psis[a], -1) for a in range(nc)])
    Ml, Mr = moment_matrix(gl, psis), moment_matrix(gr, psis)
    al = [np.linalg.solve(Ml, np.asarray(dWl[d]) / gl.rho) for d in range(D)]
    ar = [np.linalg.solve(Mr, np.asarray(dWr[d]) / gr.rho) for d in range(D)]
    dW0 = np.zeros((D, nc))
    for d in range(D):
        fl, fr = micro_fn(al[d], psis), micro_fn(ar[d], psis)
        for a in range(nc):
            dW0[d, a] = (gl.rho * gl.expect(lambda *u, a=a: psis[a](*u) * fl(*u), +1)
                         + gr.rho * gr.expect(lambda *u, a=a: psis[a](*u) * fr(*u), -1))
    g0 = Gauss(W0, D, gamma)
    M0 = moment_matrix(g0, psis)
    ab = [np.linalg.solve(M0, dW0[d] / g0.rho) for d in range(D)]

    def ua(coefs):
        fns = [micro_fn(c, psis) for c in coefs]
        return lambda u1, u2, u3, x: sum(vel(d)(u1, u2, u3, x) * fns[d](u1, u2, u3, x) for d in range(D))

    ua0, ual, uar = ua(ab), ua(al), ua(ar)
    Ab = np.linalg.solve(M0, -np.array([g0.expect(lambda *u, a=a: psis[a](*u) * ua0(*u), 0) for a in range(nc)]))
    Al = np.linalg.solve(Ml, -np.array([gl.expect(lambda *u, a=a: psis[a](*u) * ual(*u), 0) for a in range(nc)]))
    Ar = np.linalg.solve(Mr, -np.array([gr.expect(lambda *u, a=a: psis[a](*u) * uar(*u), 0) for a in range(nc)]))
    fAb, fAl, fAr = micro_fn(Ab, psis), micro_fn(Al, psis), micro_fn(Ar, psis)

    jump = abs(gl.p - gr.p) / (gl.p + gr.p)
    if tau_mode == "zero":
        tau = 0.0
    elif tau_mode == "viscous":
        tau = mu / g0.p + c2 * jump * dt
    else:
        tau = c1 * dt + c2 * jump * dt

    weights = [lambda *u, a=a: vel(0)(*u) * psis[a](*u) for a in range(nc)]
    ns = mu > 0.0 and prandtl != 1.0
    if ns:
        U0 = np.zeros(3)
        U0[:D] = g0.U

        def heat(u1, u2, u3, x):
            s = (u1 - U0[0]) ** 2 + x
            if D >= 2:
                s = s + (u2 - U0[1]) ** 2
            if D >= 3:
                s = s + (u3 - U0[2]) ** 2
            return 0.5 * (u1 - U0[0]) * s

        weights.append(heat)

    # velocity moments of each time-factor term of Eq. 2.5
    V = []
    for w in weights:
        V.append([
            g0.rho * g0.expect(w, 0),
            g0.rho * g0.expect(lambda *u, w=w: w(*u) * ua0(*u), 0),
            g0.rho * g0.expect(lambda *u, w=w: w(*u) * fAb(*u), 0),
            gl.rho * gl.expect(w, +1) + gr.rho * gr.expect(w, -1),
            gl.rho * gl.expect(lambda *u, w=w: w(*u) * ual(*u), +1) + gr.rho * gr.expect(lambda *u, w=w: w(*u) * uar(*u), -1),
            gl.rho * gl.expect(lambda *u, w=w: w(*u) * fAl(*u), +1) + gr.rho * gr.expect(lambda *u, w=w: w(*u) * fAr(*u), -1),
        ])

    def factors(t):
        if tau == 0.0:
            e = 0.0
            return [1.0, 0.0, t, 0.0, 0.0, 0.0]
        e = math.exp(-t / tau)
        return [1 - e, (t + tau) * e - tau, t - tau + tau * e, e, -(tau + t) * e, -tau * e]

    F = np.zeros((len(deltas), nc))
    for i, dl in enumerate(deltas):
        C = [integrate.quad(lambda t, k=k: factors(t)[k], 0.0, dl, epsabs=0.0, epsrel=1e-13, limit=200)[0]
             for k in range(6)]
        Fa = [sum(C[k] * V[a][k] for k in range(6)) for a in range(len(weights))]
        if ns:
            Fa[nc - 1] += (1.0 / prandtl - 1.0) * Fa[nc]
        F[i] = Fa[:nc]
    return F, W0, dW0, tau
