"""Coefficients of the device's complementary error function (tgks_device.hpp,
erfc_exp): the polynomial in y in [-1, 1] that approximates

    f(y) = (1 + 2 t) exp(t^2) erfc(t),   t = K (1 + y) / (1 - y),  K = 3.75,

(the form of M. M. Shepherd and J. G. Laframboise, "Chebyshev approximation
of (1 + 2x) exp(x^2) erfc x in 0 <= x < infinity", Math. Comp. 36 (1981)):
its Chebyshev series, computed here from the definition with mpmath (40
digits, Gauss-Chebyshev quadrature on 256 nodes), cut after 23 terms and
converted to powers of y at 40 digits.  The power coefficients are small
(sum of magnitudes 1.76), so Horner's rule in double loses nothing: in the
device's order, f(y) / (1 + 2t) is within 5.6e-16 of exp(t^2) erfc(t)
(relative) for t in [0, 27], checked below.

    python -m paper_2309_10534_amd.erfc_coeffs      # prints the C++ table
"""
import mpmath as mp

K = mp.mpf("3.75")
N = 23


def chebyshev(n=N, nodes=256):
    mp.mp.dps = 40
    ys = [mp.cos(mp.pi * (j + mp.mpf(1) / 2) / nodes) for j in range(nodes)]

    def f(y):
        t = K * (1 + y) / (1 - y)
        return (1 + 2 * t) * mp.erfc(t) * mp.exp(t * t)

    vals = [f(y) for y in ys]
    cs = []
    for k in range(n):
        s = mp.fsum(v * mp.cos(k * mp.pi * (j + mp.mpf(1) / 2) / nodes) for j, v in enumerate(vals))
        cs.append(2 * s / nodes)
    cs[0] /= 2
    return cs


def powers(cs):
    """sum c_k T_k(y) as sum a_j y^j (T_{k+1} = 2 y T_k - T_{k-1})."""
    T = [[mp.mpf(1)], [mp.mpf(0), mp.mpf(1)]]
    for k in range(2, len(cs)):
        a = [mp.mpf(0)] + [2 * x for x in T[k - 1]]
        b = T[k - 2] + [mp.mpf(0)] * (len(a) - len(T[k - 2]))
        T.append([x - y for x, y in zip(a, b)])
    out = [mp.mpf(0)] * len(cs)
    for k, ck in enumerate(cs):
        for j, t in enumerate(T[k]):
            out[j] += ck * t
    return [float(a) for a in out]


def evaluate(t, a, k=float(K)):
    """exp(t^2) erfc(t) from the polynomial, in the device's order (t >= 0):
    even and odd powers as two Horner chains in z = y^2."""
    q, s = t + k, 2.0 * t + 1.0
    r = 1.0 / (q * s)
    y = ((t - k) * s) * r
    w = q * r
    z = y * y
    ev = a[22]
    for j in range(20, -1, -2):
        ev = ev * z + a[j]
    od = a[21]
    for j in range(19, 0, -2):
        od = od * z + a[j]
    return (od * y + ev) * w


def max_error(a):
    import numpy as np
    ts = np.concatenate([np.linspace(0.0, 1.0, 1001), np.linspace(1.0, 6.0, 2001), np.geomspace(6.0, 27.0, 500)])
    mp.mp.dps = 40
    ref = [mp.erfc(mp.mpf(t)) * mp.exp(mp.mpf(t) ** 2) for t in ts]
    return max(abs(evaluate(float(t), a) / float(r) - 1.0) for t, r in zip(ts, ref))


if __name__ == "__main__":
    a = powers(chebyshev())
    print("// max relative error %.2e, sum |a_j| %.3f" % (max_error(a), sum(abs(x) for x in a)))
    print("constexpr double ERFC_POLY[%d] = {" % len(a))
    for i in range(0, len(a), 3):
        print("    " + ", ".join("%.17g" % x for x in a[i:i + 3]) + ",")
    print("};")
