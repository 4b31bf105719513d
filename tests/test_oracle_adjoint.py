"""Pins of the oracle's adjoint and spin derivative (CPU).

* dot-product identity: Re<A v, w> = Re<v, A^H w> for random complex v, w
  (complex inner product <x, y> = sum conj(x) y), for one step and for the
  bilinear extraction;
* the forward-mode tangent dA/da against Richardson-extrapolated central
  differences of the step in a;
* the whole reverse pass against finite differences of a loss
  L = sum_n |E Phi^n - y_n|^2: central differences in the initial data are
  exact up to rounding (L is quadratic in the data), differences in a are
  Richardson-extrapolated;
* the forward-mode evolution of v = du/da: its series derivative against
  Richardson-extrapolated differences of the series in a, and its dL/da
  against the reverse pass (two exact routes to one number).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1010_3816_amd import inputs


def inner(x, y):
    return np.vdot(x, y)  # sum conj(x) * y


@pytest.mark.parametrize("a,s,m,nr,nth", [(0.0, -2, 2, 40, 8), (0.7, -2, 1, 33, 7), (0.95, 0, -3, 50, 12),
                                          (0.5, 1, 0, 3, 2)])
def test_step_dot_product(a, s, m, nr, nth):
    g = oracle.OracleGrid(a, s, m, nr, nth, -20.0, 30.0, 0.03)
    v = inputs.random_state(nr, nth, 1)
    w = inputs.random_state(nr, nth, 2)
    Av = g.step(*v, 1)
    AHw = g.adjoint_step(*w)
    lhs = inner(Av[0], w[0]) + inner(Av[1], w[1])
    rhs = inner(v[0], AHw[0]) + inner(v[1], AHw[1])
    assert abs(lhs.real - rhs.real) <= 1e-13 * (abs(lhs) + 1.0)
    # complex linearity makes the full complex inner products agree as well
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + 1.0)


@pytest.mark.parametrize("m", [2, 3])
def test_extract_dot_product(m):
    g = oracle.OracleGrid(0.3, -2, m, 30, 9, -10.0, 20.0, 0.01)
    rng = np.random.default_rng(m)
    v = rng.standard_normal((9, 30)) + 1j * rng.standard_normal((9, 30))
    for rs, th in [(3.3, 1.2), (-10.0, 0.0), (20.0, math.pi), (7.7, 0.05)]:
        gv = 0.3 - 0.8j
        lhs = np.conj(g.extract(v, rs, th)) * gv
        ET = g.extract_adjoint(np.zeros((9, 30)), rs, th, gv)
        rhs = inner(v, ET)
        assert abs(lhs - rhs) <= 1e-14 * (abs(lhs) + 1.0)


@pytest.mark.parametrize("a,s,m", [(0.3, -2, 2), (0.8, 0, -1), (0.002, -2, 1)])
def test_tangent_matches_finite_differences(a, s, m):
    nr, nth = 30, 6
    u = inputs.random_state(nr, nth, 3)
    t = oracle.OracleGrid(a, s, m, nr, nth, -15.0, 25.0, 0.05).tangent_a(*u)

    def cd(h):
        up = oracle.OracleGrid(a + h, s, m, nr, nth, -15.0, 25.0, 0.05).step(*u, 1)
        um = oracle.OracleGrid(a - h, s, m, nr, nth, -15.0, 25.0, 0.05).step(*u, 1)
        return [(x - y) / (2 * h) for x, y in zip(up, um)]

    h = 1e-3
    c1, c2 = cd(h), cd(h / 2)
    rich = [(4 * y - x) / 3 for x, y in zip(c1, c2)]
    for k in range(2):
        scale = np.max(np.abs(t[k])) + 1e-300
        assert np.max(np.abs(rich[k] - t[k])) <= 1e-7 * scale


def _loss_and_grad_setup(a=0.6, s=-2, m=2, nr=60, nth=8, n=30):
    w = dict(a=a, s=s, m=m, nr=nr, nth=nth, rmin=-20.0, rmax=30.0, dt=0.05, n=n,
             er=[5.0, 12.5], et=[math.pi / 2, 1.1])
    phi0, pi0 = inputs.gaussian_pulse(nr, nth, -20.0, 30.0, 3.0, 2.0, "regular", m, s)
    rnd = inputs.random_state(nr, nth, 5)
    phi0 = phi0 + 0.1 * rnd[0]
    pi0 = pi0 + 0.1 * rnd[1]
    rng = np.random.default_rng(8)
    target = rng.standard_normal((n, 2)) * 0.01 + 1j * rng.standard_normal((n, 2)) * 0.01
    return w, phi0, pi0, target


def _loss(w, a, phi0, pi0, target):
    g = oracle.OracleGrid(a, w["s"], w["m"], w["nr"], w["nth"], w["rmin"], w["rmax"], w["dt"])
    p, q = g.project(phi0, pi0)
    _, _, ser = g.evolve(p, q, w["n"], w["er"], w["et"])
    return float(np.sum(np.abs(ser - target) ** 2)), ser


def test_reverse_pass_initial_data_gradient():
    w, phi0, pi0, target = _loss_and_grad_setup()
    L0, ser = _loss(w, w["a"], phi0, pi0, target)
    g = oracle.OracleGrid(w["a"], w["s"], w["m"], w["nr"], w["nth"], w["rmin"], w["rmax"], w["dt"])
    gser = 2.0 * (ser - target)                  # dL/dseries, PyTorch complex convention
    lp, lq, _ = g.adjoint_evolve(phi0, pi0, w["n"], w["er"], w["et"], gser)
    rng = np.random.default_rng(12)
    for _ in range(3):
        dp = rng.standard_normal(phi0.shape) + 1j * rng.standard_normal(phi0.shape)
        dq = rng.standard_normal(pi0.shape) + 1j * rng.standard_normal(pi0.shape)
        eps = 1e-3
        Lp, _ = _loss(w, w["a"], phi0 + eps * dp, pi0 + eps * dq, target)
        Lm, _ = _loss(w, w["a"], phi0 - eps * dp, pi0 - eps * dq, target)
        fd = (Lp - Lm) / (2 * eps)
        adj = float(np.real(inner(lp, dp) + inner(lq, dq)))
        assert abs(fd - adj) <= 1e-8 * max(abs(fd), 1e-12), (fd, adj)


def test_reverse_pass_spin_gradient():
    w, phi0, pi0, target = _loss_and_grad_setup()
    L0, ser = _loss(w, w["a"], phi0, pi0, target)
    g = oracle.OracleGrid(w["a"], w["s"], w["m"], w["nr"], w["nth"], w["rmin"], w["rmax"], w["dt"])
    _, _, dLda = g.adjoint_evolve(phi0, pi0, w["n"], w["er"], w["et"], 2.0 * (ser - target))

    def cd(h):
        return (_loss(w, w["a"] + h, phi0, pi0, target)[0] - _loss(w, w["a"] - h, phi0, pi0, target)[0]) / (2 * h)

    h = 1e-3
    rich = (4 * cd(h / 2) - cd(h)) / 3
    assert abs(rich - dLda) <= 1e-6 * abs(dLda), (rich, dLda)


def test_forward_mode_spin_derivative():
    """v = du/da carried forward: ds/da matches Richardson differences of the
    series in a, dL/da = sum Re(conj(dL/ds) ds/da) matches the reverse pass,
    and the state and series are those of evolve()."""
    w, phi0, pi0, target = _loss_and_grad_setup()
    L0, ser = _loss(w, w["a"], phi0, pi0, target)
    g = oracle.OracleGrid(w["a"], w["s"], w["m"], w["nr"], w["nth"], w["rmin"], w["rmax"], w["dt"])
    p, q = g.project(phi0, pi0)
    z = np.zeros_like(p)
    p1, q1, vp, vq, ser_f, tser = g.evolve_spin_tangent(p, q, z, z, w["n"], w["er"], w["et"])
    p2, q2, ser2 = g.evolve(p, q, w["n"], w["er"], w["et"])
    assert np.array_equal(p1, p2) and np.array_equal(q1, q2) and np.array_equal(ser_f, ser2)

    def ser_at(a):
        o = oracle.OracleGrid(a, w["s"], w["m"], w["nr"], w["nth"], w["rmin"], w["rmax"], w["dt"])
        pp, qq = o.project(phi0, pi0)
        return o.evolve(pp, qq, w["n"], w["er"], w["et"])[2]

    h = 1e-3
    c1 = (ser_at(w["a"] + h) - ser_at(w["a"] - h)) / (2 * h)
    c2 = (ser_at(w["a"] + h / 2) - ser_at(w["a"] - h / 2)) / h
    rich = (4 * c2 - c1) / 3
    assert np.max(np.abs(rich - tser)) <= 1e-7 * np.max(np.abs(tser))

    gser = 2.0 * (ser - target)
    _, _, dlda_rev = g.adjoint_evolve(phi0, pi0, w["n"], w["er"], w["et"], gser)
    dlda_fwd = float(np.sum(gser.real * tser.real + gser.imag * tser.imag))
    assert abs(dlda_fwd - dlda_rev) <= 1e-12 * abs(dlda_rev), (dlda_fwd, dlda_rev)


def test_forward_mode_carries_v():
    """A nonzero v^0 is carried by the homogeneous part: with u^0 = 0 the
    tangent term vanishes and v evolves by the step itself."""
    g = oracle.OracleGrid(0.7, -2, 2, 40, 8, -20.0, 30.0, 0.03)
    v = g.project(*inputs.random_state(40, 8, 21))
    z = np.zeros_like(v[0])
    _, _, vp, vq, _, _ = g.evolve_spin_tangent(z, z, v[0], v[1], 5)
    ep, eq = g.step(v[0], v[1], 5)
    assert np.array_equal(vp, ep) and np.array_equal(vq, eq)
