"""Pins of the oracle's Kerr geometry and coefficients (CPU).

* The coefficients of the first-order system are re-derived symbolically from
  Eq. (1) of arXiv:1010.3816 (typed here from the paper, with
  Psi = exp(i m phi) r^3 Phi as in Sec. 3.2) and compared with the oracle's
  values at random points.  A dropped term, a wrong sign or a wrong power in
  any coefficient fails this test.
* The tortoise inversion is checked by its round trip and by
  d(r*)/dr = (r^2 + a^2)/Delta, the defining property of r*.
* The d/da values (complex step) are checked against Richardson-extrapolated
  central differences.
"""
import math

import numpy as np
import pytest
import sympy as sp

import oracle


def _derived_coefficients(a_val, s_val, m_val):
    """Coefficients of Phi_tt, Phi'', Phi', Phi_t, Phi_thth, Phi_th, Phi in
    Eq. (1) multiplied by -Delta/(Sigma^2 r^3), as sympy expressions in (r, th);
    ' = d/dr* with d(r*)/dr = (r^2 + a^2)/Delta."""
    t, r, th = sp.symbols("t r theta", real=True)
    a = sp.nsimplify(a_val)
    s = sp.Integer(s_val)
    m = sp.Integer(m_val)
    I = sp.I
    F = sp.Function("Phi")(t, r, th)
    Delta = r**2 - 2 * r + a**2
    Psi = r**3 * F
    # Eq. (1), M = 1, acting on exp(i m phi) Psi: d_phi -> i m, d_phiphi -> -m^2
    E = (-((r**2 + a**2) ** 2 / Delta - a**2 * sp.sin(th) ** 2) * sp.diff(Psi, t, 2)
         - (4 * a * r / Delta) * (I * m) * sp.diff(Psi, t)
         - 2 * s * (r - (r**2 - a**2) / Delta + I * a * sp.cos(th)) * sp.diff(Psi, t)
         + Delta ** (-s) * sp.diff(Delta ** (s + 1) * sp.diff(Psi, r), r)
         + 1 / sp.sin(th) * sp.diff(sp.sin(th) * sp.diff(Psi, th), th)
         + (1 / sp.sin(th) ** 2 - a**2 / Delta) * (-m**2) * Psi
         + 2 * s * (a * (r - 1) / Delta + I * sp.cos(th) / sp.sin(th) ** 2) * (I * m) * Psi
         - (s**2 * sp.cot(th) ** 2 - s) * Psi)
    syms = sp.symbols("Ftt Frr Fr Ft Fhh Fh F0")
    Ftt, Frr, Fr, Ft, Fhh, Fh, F0 = syms
    E = E.subs({sp.Derivative(F, (t, 2)): Ftt, sp.Derivative(F, (r, 2)): Frr,
                sp.Derivative(F, (th, 2)): Fhh})
    E = E.subs({sp.Derivative(F, t): Ft, sp.Derivative(F, r): Fr, sp.Derivative(F, th): Fh})
    E = E.subs(F, F0)
    Sig2 = (r**2 + a**2) ** 2 - a**2 * Delta * sp.sin(th) ** 2
    E = sp.expand(E * (-Delta / (Sig2 * r**3)))
    coef = {k: E.coeff(v) for k, v in zip(("tt", "rr", "r", "t", "hh", "h", "0"), syms)}
    jac = (r**2 + a**2) / Delta          # d(r*)/dr
    out = {
        "tt": coef["tt"],
        "ss": coef["rr"] * jac**2,                          # coefficient of Phi''
        "s": coef["r"] * jac + coef["rr"] * sp.diff(jac, r),  # coefficient of Phi'
        "t": coef["t"],
        "hh": coef["hh"],
        "h": coef["h"],
        "0": coef["0"],
    }
    return {k: sp.lambdify((r, th), v, "mpmath") for k, v in out.items()}


def _num(f, r, th):
    import mpmath

    mpmath.mp.dps = 40
    return complex(f(mpmath.mpf(r), mpmath.mpf(th)))


CASES = [
    (0.0, -2, 2, 7.5, 1.1),
    (0.0, 0, 0, 25.0, 0.4),
    (0.35, -1, 3, 3.0, 2.2),
    (0.7, -2, 2, 12.0, 0.9),
    (0.7, 2, -1, 40.0, 2.9),
    (0.9, -2, -2, 1.5, 1.6),
    (0.95, 1, 1, 60.0, 0.3),
    (0.99, 0, 4, 5.0, 2.6),
]


@pytest.mark.parametrize("a,s,m,rstar,theta", CASES)
def test_coefficients_match_eq1(a, s, m, rstar, theta):
    val, _ = oracle.coefficients(a, s, m, rstar, theta)
    b, c = val[0], val[1] + 1j * val[2]
    ct = val[3] + 1j * val[4]
    a2, a1 = val[5], val[6]
    v0 = val[7] + 1j * val[8]
    x = oracle.tortoise_x(a, rstar)
    r = 1.0 + math.sqrt(1.0 - a * a) + x
    d = _derived_coefficients(a, s, m)
    assert abs(_num(d["tt"], r, theta) - 1.0) < 1e-14
    # Phi'' coefficient is -b^2, Phi_t is Ct, Phi_thth is -A2, Phi_th is -A1, Phi is V0
    assert b > 0
    assert abs(-_num(d["ss"], r, theta) - b * b) <= 1e-13 * b * b
    assert abs(_num(d["t"], r, theta) - ct) <= 1e-13 * max(1.0, abs(ct))
    assert abs(-_num(d["hh"], r, theta) - a2) <= 1e-13 * abs(a2)
    assert abs(-_num(d["h"], r, theta) - a1) <= 1e-13 * max(abs(a1), abs(a2))
    assert abs(_num(d["0"], r, theta) - v0) <= 1e-12 * max(1.0, abs(v0))
    # Phi' coefficient is -B1 with c = b b' - b Ct - B1; b' by a 4th-order
    # central difference of the oracle's b in r*.
    h = 1e-3
    bs = [oracle.coefficients(a, s, m, rstar + k * h, theta)[0][0] for k in (-2, -1, 1, 2)]
    bp = (bs[0] - 8 * bs[1] + 8 * bs[2] - bs[3]) / (12 * h)
    B1 = -_num(d["s"], r, theta)
    c_expect = b * bp - b * ct - B1
    assert abs(c - c_expect) <= 1e-8 * max(1.0, abs(c))


@pytest.mark.parametrize("a", [0.0, 0.3, 0.7, 0.9, 0.99])
def test_tortoise_round_trip(a):
    rp = 1 + math.sqrt(1 - a * a)
    rm = 1 - math.sqrt(1 - a * a)
    d = rp - rm
    for rs in np.linspace(-200.0, 1200.0, 701):
        x = oracle.tortoise_x(a, rs)
        assert x > 0.0
        back = oracle.rstar_of_x(a, x)
        # the evaluation of r*(x) itself rounds at the scale of its largest term
        scale = max(abs(rp + x), abs(2 * rp / d * math.log(x / 2)),
                    abs(2 * rm / d * math.log((x + d) / 2)), abs(rs))
        assert abs(back - rs) <= 4 * np.spacing(scale)


@pytest.mark.parametrize("a", [0.0, 0.5, 0.99])
@pytest.mark.parametrize("rs", [-200.0, -60.0, -5.0, 3.0, 50.0, 900.0])
def test_tortoise_derivative(a, rs):
    """d(ln x)/dr* = Delta/(x (r^2 + a^2)) = (x + r+ - r-)/(r^2 + a^2)."""
    h = 1e-4
    xs = [oracle.tortoise_x(a, rs + k * h) for k in (-2, -1, 1, 2)]
    ly = [math.log(v) for v in xs]
    dlnx = (ly[0] - 8 * ly[1] + 8 * ly[2] - ly[3]) / (12 * h)
    x = oracle.tortoise_x(a, rs)
    rp = 1 + math.sqrt(1 - a * a)
    rm = 1 - math.sqrt(1 - a * a)
    r = rp + x
    expect = (x + rp - rm) / (r * r + a * a)
    assert abs(dlnx - expect) <= 1e-8 * abs(expect)


def test_delta_positive_near_horizon():
    for a in (0.0, 0.7, 0.99):
        x = oracle.tortoise_x(a, -200.0)
        assert 0.0 < x < 1e-10
        rp = 1 + math.sqrt(1 - a * a)
        rm = 1 - math.sqrt(1 - a * a)
        assert x * (x + rp - rm) > 0.0


@pytest.mark.parametrize("a,s,m,rstar,theta", [(0.3, -2, 2, 4.0, 1.0), (0.7, 0, -3, -20.0, 2.5),
                                                (0.9, -2, 1, 30.0, 0.2)])
def test_coefficient_a_derivative(a, s, m, rstar, theta):
    """Complex-step d/da against Richardson-extrapolated central differences."""
    _, dval = oracle.coefficients(a, s, m, rstar, theta)

    def cd(h):
        vp, _ = oracle.coefficients(a + h, s, m, rstar, theta)
        vm, _ = oracle.coefficients(a - h, s, m, rstar, theta)
        return (vp - vm) / (2 * h)

    h = 1e-3
    rich = (4 * cd(h / 2) - cd(h)) / 3
    scale = np.maximum(np.abs(dval), 1.0)
    assert np.all(np.abs(rich - dval) <= 1e-7 * scale)
