"""The double Mach reflection's initial field (input generation, Sec. 5.7):
exact area fractions of the cells cut by the 60-degree shock against
brute-force point sampling, the two states on either side, and the boundary
description's shock line moving at the shock's horizontal speed."""
import math

import numpy as np

from paper_2309_10534_amd import inputs as I


def test_cut_cell_fractions_against_sampling():
    nx, ny = 48, 12
    W, (dx, dy), spec = I.double_mach(nx, ny)
    A, B = np.array(spec["states"][0]), np.array(spec["states"][1])
    # fraction of state A in each cell from the density
    f = (W[0] - B[0]) / (A[0] - B[0])
    m = 200
    rng = np.random.default_rng(0)
    for j, i in [(0, 3), (0, 4), (5, 6), (11, 9), (7, 7)] + [tuple(x) for x in rng.integers(0, [ny, nx], (10, 2))]:
        xs = (i + (np.arange(m) + 0.5) / m) * dx
        ys = (j + (np.arange(m) + 0.5) / m) * dy
        X, Y = np.meshgrid(xs, ys)
        exact = np.mean(X < 1.0 / 6.0 + Y / math.sqrt(3.0))
        assert abs(f[j, i] - exact) < 2e-4, (j, i, f[j, i], exact)
    # every component mixes with the same fraction
    for c in range(4):
        assert np.allclose(W[c], f * A[c] + (1 - f) * B[c], rtol=0, atol=1e-12)


def test_states_and_line():
    W, (dx, dy), spec = I.double_mach(96, 24)
    A, B = spec["states"]
    rho, (u, v), p = I.primitive(np.array(A).reshape(4, 1, 1))
    assert abs(rho.item() - 8.0) < 1e-14 and abs(p.item() - 116.5) < 1e-12
    assert abs(u.item() - 4.125 * math.sqrt(3.0)) < 1e-14 and abs(v.item() + 4.125) < 1e-14
    assert B[:3] == [1.4, 0.0, 0.0] and abs(B[3] - 2.5) < 1e-14
    s0, sn, st = spec["lines"][(1, 1)]
    # the Mach 10 shock moves at 10 along its normal (cos 30, -sin 30), i.e.
    # at 10 / cos 30 = 20 / sqrt 3 along x; the line at y has x = s0 + sn y
    assert abs(s0 - 1.0 / 6.0) < 1e-15 and abs(sn - math.tan(math.pi / 6)) < 1e-15
    assert abs(st - 10.0 / math.cos(math.pi / 6)) < 1e-13
    assert spec["far"][(1, 0)] == "reflective" and spec["lines"][(1, 0)] == (1.0 / 6.0, 0.0, 0.0)
