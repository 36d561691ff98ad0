"""The device Gauss-point flux (closed-form moments, Jacobian-vector
products of the Euler flux and of the second-moment flux, closed-form
micro-slope solves), evaluated on the host through tgks_gp_flux_host, against
the oracle's generic moment engine.  No device needed."""
import os

import numpy as np
import pytest

from paper_2309_10534_amd.inputs import conservative


@pytest.fixture(scope="module")
def tg():
    from paper_2309_10534_amd import tgks
    if not os.path.exists(tgks.LIB_PATH):
        pytest.skip("libtgks.so not built")
    return tgks


def rand_state(rng, D):
    return conservative(np.array([rng.uniform(0.3, 3.0)]), [np.array([rng.uniform(-1.5, 1.5)]) for _ in range(D)],
                        np.array([rng.uniform(0.2, 3.0)]))[:, 0]


@pytest.mark.parametrize("D", [1, 2, 3])
@pytest.mark.parametrize("mode", ["inviscid", "viscous", "zero"])
def test_device_flux_matches_oracle(orc, tg, D, mode):
    rng = np.random.default_rng(7 + D + len(mode))
    mu, pr = (0.05, 0.72) if mode == "viscous" else (0.0, 1.0)
    P = orc.make_params([8] * D, [0.1] * D, tau=mode, mu=mu, prandtl=pr)
    Pg = tg.tgks_params_default(D, [8] * D, [0.1] * D, tau=mode, mu=mu, prandtl=pr)
    for _ in range(20):
        Wl, Wr = rand_state(rng, D), rand_state(rng, D)
        dWl = rng.normal(size=(D, D + 2)) * 0.5
        dWr = rng.normal(size=(D, D + 2)) * 0.5
        dt = rng.uniform(1e-3, 0.05)
        Fo, _, _, bad = orc.gp_flux(P, Wl, Wr, dWl, dWr, dt, [dt, dt / 2])
        Fg, ok = tg.tgks_gp_flux_host(Pg, Wl, Wr, dWl, dWr, dt)
        assert ok and bad == 0
        np.testing.assert_allclose(Fg, Fo, rtol=1e-12, atol=1e-13 * np.abs(Fo).max())


def test_device_flux_flags_nonphysical(tg):
    Pg = tg.tgks_params_default(1, [8], [0.1])
    good = conservative(np.array([1.0]), [np.array([0.2])], np.array([1.0]))[:, 0]
    bad = good.copy()
    bad[2] = -1.0
    assert tg.tgks_gp_flux_host(Pg, good, good, np.zeros(3), np.zeros(3), 0.01)[1]
    assert not tg.tgks_gp_flux_host(Pg, good, bad, np.zeros(3), np.zeros(3), 0.01)[1]


def stencils(rng, n):
    """Five-value stencils of every kind the selection meets: smooth, jumps,
    constants (exact and with last-bit noise), linear ramps, huge and tiny
    magnitudes, NaN and infinity."""
    out = []
    for i in range(n):
        k = i % 9
        if k == 0:
            Q = rng.normal(size=5)
        elif k == 1:
            Q = 1.0 + 0.01 * np.sin(rng.uniform(0, 6) + 0.2 * np.arange(5))
        elif k == 2:
            Q = np.where(np.arange(5) < rng.integers(1, 5), 1.0, 0.1) + 1e-4 * rng.normal(size=5)
        elif k == 3:
            Q = np.full(5, rng.choice([0.7, 1.0, 3.3]))
        elif k == 4:
            Q = np.full(5, 0.7) * (1 + rng.choice([0.0, 1.1e-16, -2.2e-16], size=5))
        elif k == 5:
            Q = rng.uniform(-1, 1) + rng.uniform(-1, 1) * np.arange(5.0)
        elif k == 6:
            Q = rng.normal(size=5) * 10.0 ** rng.uniform(-30, 30)
        elif k == 7:
            Q = 1.0 + rng.normal(size=5) * 10.0 ** rng.integers(-8, -2)
        else:
            Q = rng.normal(size=5)
            Q[rng.integers(0, 5)] = rng.choice([np.nan, np.inf, -np.inf, 1e200])
        out.append(Q)
    return out


@pytest.mark.parametrize("ct1,ct2,eps", [(1e-7, 1e-5, 1e-40), (1e-5, 1e-6, 1e-40), (1e-7, 2e-6, 1e-6),
                                         (0.25, 1e-5, 1e-40), (1e-7, 0.3, 1e-40), (1e-7, 1e-5, 1e-300)])
def test_teno_flag_shortcut_is_exact(orc, ct1, ct2, eps):
    """The kernels decide certain selections with less work than the
    weights of Eq. 4.5 by correctly rounded divisions: the 3-D kernels from
    ratios of b_3 and b_k to min b_k derived from C_T1, C_T2, the 1-D and
    2-D kernels from approximate reciprocals with a margin.  Over
    stencils of every kind each flag equals the one from the exact weights
    bit for bit, and all equal the oracle's selection (finite inputs).
    Constants with last-bit noise reject the large stencil, smooth data
    keep it."""
    from paper_2309_10534_amd import tgks
    p = tgks.tgks_params_default(1, [10], [0.1])
    p.ct1, p.ct2, p.eps = ct1, ct2, eps
    rng = np.random.default_rng(7)
    seen = set()
    for Q in stencils(rng, 20000):
        a = tgks.tgks_teno_flag_host(p, Q, fast=1)
        b = tgks.tgks_teno_flag_host(p, Q, fast=0)
        c = tgks.tgks_teno_flag_host(p, Q, fast=2)
        assert a == b == c, Q
        if np.all(np.isfinite(Q)):
            assert a == orc.teno_select(Q, ct1=ct1, ct2=ct2, eps=eps), Q
        seen.add(a)
    assert 1 in seen and 14 in seen and len(seen) >= 4, seen


@pytest.mark.parametrize("ct1,ct2", [(1e-7, 1e-5), (1e-5, 1e-6), (0.2, 0.2)])
def test_teno_flag_shortcut_at_decision_boundaries(ct1, ct2):
    """Along segments between stencils of different flags, the point where
    the weights' decision changes is found by bisection to the last bit;
    at every stencil within a few ulps of it on either side both shortcuts
    return the weights' flag (they never claim a decision that rounding or
    an approximate reciprocal could flip)."""
    from paper_2309_10534_amd import tgks
    p = tgks.tgks_params_default(1, [10], [0.1])
    p.ct1, p.ct2 = ct1, ct2
    rng = np.random.default_rng(11)
    flag = lambda Q, fast: tgks.tgks_teno_flag_host(p, Q, fast=fast)
    found = 0
    for _ in range(300):
        A = rng.normal(size=5) * 10.0 ** rng.uniform(-3, 1)
        B = A.copy()
        B[rng.integers(0, 5)] += rng.normal() * 10.0 ** rng.uniform(-3, 1)
        fa, fb = flag(A, False), flag(B, False)
        if fa == fb:
            continue
        lo, hi = 0.0, 1.0
        for _ in range(70):
            mid = 0.5 * (lo + hi)
            if mid in (lo, hi):
                break
            if flag(A + mid * (B - A), False) == fa:
                lo = mid
            else:
                hi = mid
        found += 1
        t = lo
        for _ in range(8):
            t = np.nextafter(t, -1.0)
        ts = []
        for _ in range(16):
            ts.append(t)
            t = np.nextafter(t, 2.0)
        # and at relative distances 1e-15 .. 1e-2 from the boundary, across
        # the approximate reciprocals' error and the margin of 2^-12
        ts += [lo * (1.0 + sg * 10.0 ** -j) for j in range(2, 16) for sg in (-1.0, 1.0)]
        for t in ts:
            Q = A + t * (B - A)
            assert flag(Q, 1) == flag(Q, 0) == flag(Q, 2), (ct1, ct2, Q.tolist())
    assert found > 50


# Stencils on which each certain-decision bound is (nearly) reached, and the
# indicator that is placed at the bound relative to min(b_0, b_1, b_2):
# equal small indicators (large stencil kept), one smooth small stencil
# with two rougher ones (large stencil rejected: (0, 0, 0, 1, 4) has
# beta_3 = 1.7 beta_1 and beta_2 = 3.3 beta_1; a small one dropped), two
# equal smooth small stencils with a rougher third and a rougher quartic
# (a small one kept: (1, 0, 0, -1, -1/2) has beta_0 = beta_1 exactly,
# beta_2 = 4.1 beta_0, beta_3 = 18 beta_0, so the large stencil is
# rejected for certain at the bound).
BOUND_CASES = [
    ("keep_large", [0.75, 1.0, 0.0, 1.0, 0.75], 3, lambda c1, c2: ((1 / c1 - 1) / 3) ** (1 / 7)),
    ("reject_large", [0.0, 0.0, 0.0, 1.0, 4.0], 3, lambda c1, c2: (1 / c1 - 1) ** (1 / 7)),
    ("keep_small", [1.0, 0.0, 0.0, -1.0, -0.5], 2, lambda c1, c2: ((1 / c2 - 1) / 2) ** (1 / 7)),
    ("drop_small", [0.0, 0.0, 0.0, 1.0, 100.0], 1, lambda c1, c2: (1 / c2 - 1) ** (1 / 7)),
]


# cut-off pairs per bound: the paper's (where the stencil reaches the
# bound), the cut-off at the edge of the range in which the kernels' fixed
# ratios hold, and just outside it (shortcut off)
BOUND_CTS = {"keep_large": [(1e-7, 1e-5), (2.0e-5, 1e-5), (2.1e-5, 1e-5)],
             "reject_large": [(1e-7, 1e-5), (3.8e-9, 1e-5), (3.6e-9, 1e-5)],
             "keep_small": [(1e-7, 3.0e-5), (1e-7, 3.2e-5)],
             "drop_small": [(1e-7, 1e-5), (1e-7, 4.8e-7), (1e-7, 4.6e-7)]}
BOUND_PARAMS = [pytest.param(case, ct1, ct2, id=f"{case[0]}-{ct1:g}-{ct2:g}")
                for case in BOUND_CASES for ct1, ct2 in BOUND_CTS[case[0]]]


@pytest.mark.parametrize("case,ct1,ct2", BOUND_PARAMS)
def test_teno_flag_shortcut_at_worst_case_bounds(orc, case, ct1, ct2):
    """The selection rule (Eqs. 4.6-4.7, 4.11-4.12) on gamma_k = b_k^-7
    decides from ratios of the b_k alone at worst-case stencils: with the
    three small b equal, the large stencil is kept iff b_3 / b <=
    ((1 / C_T1 - 1) / 3)^(1/7); with one smooth small stencil and two
    infinitely rough ones, it is kept iff b_3 / m <= (1 / C_T1 - 1)^(1/7),
    and a second small stencil is kept iff b_k / m <= (1 / C_T2 - 1)^(1/7);
    with two equal smooth ones, the third is kept iff b_k / m <=
    ((1 / C_T2 - 1) / 2)^(1/7).  eps (b_k = beta_k + eps) places the ratio
    at the bound times (1 +- delta); at every point the shortcut returns the
    weights' flag and the oracle's.  At the edges of the cut-off range in
    which the kernels' ratios hold the bound lies within 0.3 % of a ratio,
    just outside the range on its wrong side: a range or ratio a little too
    wide fails here."""
    from paper_2309_10534_amd import tgks
    name, Q, k, bound = case
    Q = np.array(Q)
    be = np.asarray(orc.beta(Q), dtype=float)
    p = tgks.tgks_params_default(1, [10], [0.1])
    p.ct1, p.ct2 = ct1, ct2
    rho0 = bound(ct1, ct2)
    m = be[:3].min()
    decided = set()
    assert (be[k] - rho0 * (1 + 1e-3) * m) / (rho0 * (1 + 1e-3) - 1) > 1e-40, (name, rho0, "beyond reach")
    for delta in (-1e-3, -1e-6, -1e-9, -1e-12, 1e-12, 1e-9, 1e-6, 1e-3):
        rho = rho0 * (1 + delta)
        eps = (be[k] - rho * m) / (rho - 1)
        p.eps = eps
        a = tgks.tgks_teno_flag_host(p, Q, fast=1)
        b = tgks.tgks_teno_flag_host(p, Q, fast=0)
        c = tgks.tgks_teno_flag_host(p, Q, fast=2)
        assert a == b == c == orc.teno_select(Q, ct1=ct1, ct2=ct2, eps=eps), (name, delta, a, b, c)
        decided.add((delta > 0, b))
    # the bound separates two decisions: it is reached exactly for equal
    # small indicators and to a few parts in 1e6 (the rough stencils' own
    # gamma) for the others
    assert len({f for _, f in decided}) == 2, (name, sorted(decided))


def test_erfc_series_accuracy():
    """The kernels' erfc (the Chebyshev series of (1 + 2t) exp(t^2) erfc(t)
    in y = (t - 3.75) / (t + 3.75), cut after 23 terms and summed in powers
    of y, divided by 1 + 2t and times exp(-x^2)) against mpmath's erfc
    of the same double x at 50 digits: within 1e-15 relative, plus the
    conditioning of exp(-x^2) in x (2 x^2 ulps: the rounding of x * x),
    for |x| up to 27, where erfc(x) underflows; exact limits at +-inf and
    a NaN for a NaN.  A wrong coefficient or K, a dropped term, a skipped
    Newton step of the reciprocal or a wrong even/odd recombination fails
    here."""
    import math
    import mpmath as mp
    from paper_2309_10534_amd import tgks
    mp.mp.dps = 50
    xs = np.concatenate([np.linspace(-6.0, 6.0, 2401), np.geomspace(1e-300, 1e-3, 40),
                         -np.geomspace(1e-300, 1e-3, 40), np.geomspace(6.0, 27.0, 300), -np.geomspace(6.0, 27.0, 30),
                         [0.0, -0.0, 3.75, -3.75, 0.5, -0.5]])
    worst = 0.0
    for x in xs:
        ref = mp.erfc(mp.mpf(float(x)))
        got = tgks.tgks_erfc_host(float(x))
        tol = 1e-15 + 2.0 * x * x * 2.0 ** -53
        err = abs(got - float(ref)) / float(ref)
        worst = max(worst, err / tol)
        assert err <= tol, (x, got, float(ref), err)
    assert worst > 0.01  # the check sees the series' own rounding
    assert tgks.tgks_erfc_host(math.inf) == 0.0 and tgks.tgks_erfc_host(-math.inf) == 2.0
    assert math.isnan(tgks.tgks_erfc_host(math.nan))
    assert tgks.tgks_erfc_host(40.0) == 0.0 and tgks.tgks_erfc_host(-40.0) == 2.0
