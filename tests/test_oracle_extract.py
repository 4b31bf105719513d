"""Pin of the oracle's waveform extraction (CPU): bilinear interpolation in
(r*, theta) reproduces bilinear functions exactly between row centres, and
outside the first/last row centre follows the angular boundary condition
(zero slope at the pole for even |m|, zero value for odd |m|)."""
import math

import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("m", [2, 1])
def test_bilinear_exact_interior(m):
    g = oracle.OracleGrid(0.3, -2, m, 37, 11, -20.0, 40.0, 0.01)
    rs, th = g.rstar(), g.theta()
    f = lambda x, t: (0.7 - 0.2j) + 0.05 * x + (1.3 + 0.4j) * t - 0.02j * x * t
    phi = f(rs[None, :], th[:, None])
    rng = np.random.default_rng(3)
    for _ in range(50):
        x = rng.uniform(-20.0, 40.0)
        t = rng.uniform(th[0], th[-1])
        assert abs(g.extract(phi, x, t) - f(x, t)) < 1e-13
    # endpoints of the r* range
    assert abs(g.extract(phi, 40.0, th[3]) - f(40.0, th[3])) < 1e-13
    assert abs(g.extract(phi, -20.0, th[3]) - f(-20.0, th[3])) < 1e-13


def test_pole_ghosts():
    for m, expect_zero in ((2, False), (3, True)):
        g = oracle.OracleGrid(0.0, 0, m, 21, 8, 0.0, 20.0, 0.01)
        rng = np.random.default_rng(m)
        phi = rng.standard_normal((8, 21)) + 1j * rng.standard_normal((8, 21))
        x = 7.25
        i0 = 7
        row0 = 0.75 * phi[0, i0] + 0.25 * phi[0, i0 + 1]
        rowN = 0.75 * phi[-1, i0] + 0.25 * phi[-1, i0 + 1]
        at0 = g.extract(phi, x, 0.0)
        atpi = g.extract(phi, x, math.pi)
        if expect_zero:
            assert abs(at0) < 1e-15 and abs(atpi) < 1e-15
            # linear from zero at the pole to the row-0 value at its centre
            assert abs(g.extract(phi, x, 0.25 * g.dth) - 0.5 * row0) < 1e-14
        else:
            assert abs(at0 - row0) < 1e-14 and abs(atpi - rowN) < 1e-14
            assert abs(g.extract(phi, x, 0.25 * g.dth) - row0) < 1e-14
