"""Pins of the oracle's TENO-D reconstruction (Sec. 4.2) against what the
mathematics fixes, independently of the oracle's own formulas:

  * polynomial exactness: cell averages of random polynomials of degree <= 2
    (small stencils) and <= 4 (large stencil) must give back the exact point
    values and derivatives at x = +-1/2 and at the Gauss points +-1/(2 sqrt 3);
  * smoothness indicators: Eq. 3.7 evaluated by exact integration of the
    least-squares-free polynomial fit (numpy.polynomial) equals the oracle's
    closed forms;
  * the selection: brute force with exact rational arithmetic on integer data,
    and the special cases (constant, linear, one jump at each position).
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

SQ = 1.0 / (2.0 * math.sqrt(3.0))


def cell_averages(coef, offsets):
    """Exact averages over [j-1/2, j+1/2] of sum coef[i] x^i."""
    P = np.polynomial.Polynomial(coef)
    I = P.integ()
    return np.array([I(j + 0.5) - I(j - 0.5) for j in offsets])


def fit(Q, cells):
    """Polynomial whose cell averages over `cells` equal Q (solve the
    moment conditions of Sec. 3.1 / 3.2 directly)."""
    n = len(cells)
    A = np.zeros((n, n))
    for r, j in enumerate(cells):
        for i in range(n):
            A[r, i] = ((j + 0.5) ** (i + 1) - (j - 0.5) ** (i + 1)) / (i + 1)
    return np.polynomial.Polynomial(np.linalg.solve(A, Q))


STENCILS = {0: [-2, -1, 0], 1: [-1, 0, 1], 2: [0, 1, 2], 3: [-2, -1, 0, 1, 2]}


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_polynomial_exactness(orc, k):
    rng = np.random.default_rng(10 + k)
    deg = 4 if k == 3 else 2
    flag = 1 if k == 3 else (2 << k)
    for _ in range(20):
        coef = rng.normal(size=deg + 1)
        P = np.polynomial.Polynomial(coef)
        Q = cell_averages(coef, [-2, -1, 0, 1, 2])
        face = orc.teno_eval(Q, flag, gauss=False)
        np.testing.assert_allclose(face, [P(-0.5), P.deriv()(-0.5), P(0.5), P.deriv()(0.5)],
                                   rtol=0, atol=1e-13)
        gp = orc.teno_eval(Q, flag, gauss=True)
        np.testing.assert_allclose(gp, [P(-SQ), P.deriv()(-SQ), P(SQ), P.deriv()(SQ)],
                                   rtol=0, atol=1e-13)


def test_equal_weight_combination(orc):
    # Eqs. 4.13-4.14: with d_k = 1/3 the surviving small stencils are averaged
    rng = np.random.default_rng(4)
    Q = rng.normal(size=5)
    single = {k: orc.teno_eval(Q, 2 << k) for k in range(3)}
    for mask in range(1, 8):
        ks = [k for k in range(3) if mask >> k & 1]
        got = orc.teno_eval(Q, mask << 1)
        want = sum(single[k] for k in ks) / len(ks)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-14)


def beta_quadrature(Q):
    out = []
    for k in range(4):
        cells = STENCILS[k]
        P = fit(Q[[c + 2 for c in cells]], cells)
        qk = 4 if k == 3 else 2
        s = 0.0
        for q in range(1, qk + 1):
            d = P.deriv(q)
            s += (d * d).integ()(0.5) - (d * d).integ()(-0.5)
        out.append(s)
    return np.array(out)


def test_smoothness_indicators_eq37(orc):
    rng = np.random.default_rng(7)
    for _ in range(50):
        Q = rng.normal(size=5) * rng.uniform(0.01, 100)
        np.testing.assert_allclose(orc.beta(Q), beta_quadrature(Q), rtol=1e-11, atol=1e-13 * np.max(Q ** 2))


def select_exact(Q, ct1=Fraction(1, 10 ** 7), ct2=Fraction(1, 10 ** 5), q=7):
    """Eqs. 4.5-4.12 in exact rational arithmetic, eps = 1e-40 included."""
    Qf = [Fraction(int(v)) for v in Q]
    a, b, c, d, e = Qf
    k13 = Fraction(13, 12)
    beta = [k13 * (a - 2 * b + c) ** 2 + Fraction(1, 4) * (a - 4 * b + 3 * c) ** 2,
            k13 * (b - 2 * c + d) ** 2 + Fraction(1, 4) * (b - d) ** 2,
            k13 * (c - 2 * d + e) ** 2 + Fraction(1, 4) * (3 * c - 4 * d + e) ** 2]
    P1 = (82 * (d - b) - 11 * (e - a)) / Fraction(120)
    P2 = (-3 * a + 40 * b - 74 * c + 40 * d - 3 * e) / Fraction(56)
    P3 = ((e - a) - 2 * (d - b)) / Fraction(12)
    P4 = (a - 4 * b + 6 * c - 4 * d + e) / Fraction(24)
    beta.append((P1 + P3 / 10) ** 2 + Fraction(13, 3) * (P2 + Fraction(123, 455) * P4) ** 2
                + Fraction(781, 20) * P3 ** 2 + Fraction(1421461, 2275) * P4 ** 2)
    eps = Fraction(1, 10 ** 40)
    g = [1 / (bt + eps) ** q for bt in beta]
    chi = g[3] / sum(g)
    if not chi < ct1:
        return 1, None
    s3 = g[0] + g[1] + g[2]
    f = 0
    margins = []
    for k in range(3):
        ch = g[k] / s3
        margins.append(abs(ch - ct2) / ct2)
        if not ch < ct2:
            f |= 2 << k
    return f, min(margins + [abs(chi - ct1) / ct1])


def test_selection_brute_force_exact(orc):
    rng = np.random.default_rng(11)
    checked = 0
    for _ in range(400):
        Q = rng.integers(-6, 7, size=5).astype(float)
        want, margin = select_exact(Q)
        if margin is not None and margin < 1e-9:
            continue  # decision within rounding of the threshold
        assert orc.teno_select(Q) == want, (Q, want)
        checked += 1
    assert checked > 300


def test_selection_special_cases(orc):
    # constant data whose stencil sums are exact: all beta = 0, chi = 1/4, the
    # large stencil is kept
    for c in (1.0, 0.5, -2.0, 1024.0, 0.0):
        assert orc.teno_select(np.full(5, c)) == 1
    # linear data: beta_0..3 equal the squared slope, chi = 1/4
    assert orc.teno_select(np.arange(5) * 0.3 + 1.0) == 1
    # a jump between positions j and j+1: only the stencils not crossing it survive
    for j in range(4):
        Q = np.where(np.arange(5) <= j, 1.0, 2.0)
        f = orc.teno_select(Q)
        assert f & 1 == 0
        crossing = {k for k in range(3) if STENCILS[k][0] + 2 <= j < STENCILS[k][-1] + 2}
        survivors = {k for k in range(3) if f >> (k + 1) & 1}
        assert survivors == set(range(3)) - crossing, (j, f)


def test_at_least_one_small_stencil_survives(orc):
    rng = np.random.default_rng(5)
    for _ in range(2000):
        Q = rng.normal(size=5) * 10 ** rng.uniform(-8, 8, size=5)
        f = orc.teno_select(Q)
        assert f == 1 or (f & 0b1110) != 0


def test_face_values_mirror_symmetry(orc):
    # reversing the stencil swaps the two faces and negates the slopes
    rng = np.random.default_rng(6)
    for _ in range(100):
        Q = rng.normal(size=5)
        out, f = orc.teno_face(Q)
        outr, fr = orc.teno_face(Q[::-1].copy())
        assert (f & 1) == (fr & 1)
        np.testing.assert_allclose(out, [outr[2], -outr[3], outr[0], -outr[1]], rtol=0, atol=1e-13)


def test_selection_on_roundoff_level_indicators(orc):
    """With eps = 1e-40 and q = 7 (Eq. 4.5) the selection on constant data whose
    stencil sums round (here 3.7) is decided by O(1e-30) rounding residues of
    the indicators, so the large stencil can be dropped; every candidate then
    returns the constant to rounding, so the values are unaffected."""
    Q = np.full(5, 3.7)
    b = orc.beta(Q)
    assert b.max() < 1e-28
    out, f = orc.teno_face(Q)
    np.testing.assert_allclose(out, [3.7, 0.0, 3.7, 0.0], rtol=0, atol=1e-14)
    assert f != 1


@pytest.mark.parametrize("flag", [1, 2, 4, 8, 6, 10, 12, 14])
def test_canonical_gauss_order_matches_plain_evaluation(orc, flag):
    """The 3-D first sweep evaluates the selected polynomial at the Gauss
    points in a fixed operation order (its results feed the second sweep's
    selections); on random data it equals the plain evaluation of the
    selected candidates' monomials to rounding, for the large stencil and
    every combination of surviving small stencils."""
    rng = np.random.default_rng(flag)
    for _ in range(20):
        Q = rng.normal(size=5) * 10.0 ** rng.uniform(-3, 3)
        a = orc.teno_gauss_canonical(Q, flag)
        b = orc.teno_eval(Q, flag, gauss=True)
        scale = np.abs(Q).max()
        assert np.abs(a - b).max() <= 1e-14 * scale, (flag, a, b)
