"""Pins of the oracle's inhomogeneous variant (a source J = f(t) g(r*, theta)
in the Pi equation, the form a particle-driven Teukolsky problem takes; the
paper gives no source model, so f and g are inputs).  Reading: J is part of
S's Pi row, at (t_n, r*_{i+1/2}) in stage 1 and at (t_n + dt/2, r*_i) in
stage 2.

* f = 0: exactly the homogeneous step.
* The evolution is affine in the data and linear in the source.
* Constant-coefficient wave (b = 1, the rest 0) with a uniform source F:
  Pi = F t and Phi = F t^2 / 2 exactly (the two stages integrate these
  polynomials in time exactly), away from the radial boundaries; with the
  linear profile g = r*: Pi = F (r* t + t^2/2) and Phi = F r* t^2 / 2, also
  exactly, which holds only with g taken at the half points in stage 1.
* The same wave forced by J = exp(i (w t + k r*)) from rest has the closed form
    Pi  = [e^{i(w t + k r*)} - e^{i k (r* + t)}] / (i (w - k)),
    Phi = e^{i k (r* - t)} / (i (w - k)) [ (e^{i (w + k) t} - 1)/(i (w + k))
                                          - (e^{2 i k t} - 1)/(2 i k) ];
  the oracle converges to it at second order (error ratio about 4 under
  halving dr and dt), which takes f at the times and g at the positions
  stated above: any other placement makes the scheme first order.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1010_3816_amd import inputs

NC = oracle.NCOEF


def _const_grid(nr, nth, rmin, rmax, dt, m=0, **coef):
    g = oracle.OracleGrid(0.0, 0, m, nr, nth, rmin, rmax, dt, kerr=False)
    ci = np.zeros((NC, nth, nr))
    ch = np.zeros((NC, nth, nr - 1))
    for k, v in coef.items():
        ci[oracle.COEF_NAMES.index(k)] = v
        ch[oracle.COEF_NAMES.index(k)] = v
    g.set_coefficients(ci, ch)
    return g


def _profiles(g, fn):
    x = g.rstar()
    xh = 0.5 * (x[1:] + x[:-1])
    nth = g.shape[0]
    return np.tile(fn(x), (nth, 1)), np.tile(fn(xh), (nth, 1))


def test_zero_source_is_the_homogeneous_step():
    w = dict(a=0.7, s=-2, m=2, nr=90, ntheta=14, rstar_min=-20.0, rstar_max=40.0)
    dt = inputs.stable_dt(60.0 / 89, 14, 2, -2, 50)
    o = oracle.OracleGrid(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], dt)
    p0, q0 = o.project(*inputs.random_state(90, 14, seed=1))
    rng = np.random.default_rng(2)
    o.set_source(rng.standard_normal((14, 90)) + 0j, rng.standard_normal((14, 89)) + 0j)
    a = o.evolve_source(p0, q0, np.zeros((7, 2)), [10.0], [1.0])
    b = o.evolve(p0, q0, 7, [10.0], [1.0])
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_affine_in_data_linear_in_source():
    o = oracle.OracleGrid(0.9, -2, 1, 80, 12, -20.0, 40.0, 0.01)
    rng = np.random.default_rng(3)
    gi = rng.standard_normal((12, 80)) + 1j * rng.standard_normal((12, 80))
    gh = rng.standard_normal((12, 79)) + 1j * rng.standard_normal((12, 79))
    o.set_source(gi, gh)
    f1 = rng.standard_normal((9, 2)) + 1j * rng.standard_normal((9, 2))
    f2 = rng.standard_normal((9, 2)) + 1j * rng.standard_normal((9, 2))
    p0, q0 = o.project(*inputs.random_state(80, 12, seed=4))
    z = np.zeros_like(p0)
    c = 0.4 - 1.7j
    full = o.evolve_source(p0, q0, f1 + c * f2)
    parts = [o.evolve(p0, q0, 9), o.evolve_source(z, z, f1), o.evolve_source(z, z, f2)]
    for k in range(2):
        rhs = parts[0][k] + parts[1][k] + c * parts[2][k]
        assert np.max(np.abs(full[k] - rhs)) <= 1e-12 * np.max(np.abs(rhs))


def test_uniform_source_exact_polynomials():
    nr, nth, n = 120, 6, 30
    g = _const_grid(nr, nth, -10.0, 10.0, 0.05, m=2, b=1.0)
    F = 1.3 - 0.4j
    g.set_source(*_profiles(g, lambda x: np.ones_like(x) + 0j))
    z = np.zeros(g.shape, dtype=np.complex128)
    p, q, _ = g.evolve_source(z, z, np.full((n, 2), F))
    t = n * 0.05
    inner = slice(n + 1, nr - n - 1)  # columns the zeroed radial boundaries cannot have reached
    assert np.max(np.abs(q[:, inner] - F * t)) <= 1e-13 * abs(F * t)
    assert np.max(np.abs(p[:, inner] - F * t * t / 2)) <= 1e-13 * abs(F * t * t / 2)


def test_linear_profile_exact():
    nr, nth, n, dt = 120, 4, 30, 0.05
    g = _const_grid(nr, nth, -10.0, 10.0, dt, m=2, b=1.0)
    g.set_source(*_profiles(g, lambda x: x + 0j))
    F = 0.8 + 0.3j
    z = np.zeros(g.shape, dtype=np.complex128)
    p, q, _ = g.evolve_source(z, z, np.full((n, 2), F))
    t, x, inner = n * dt, g.rstar(), slice(n + 1, nr - n - 1)
    assert np.max(np.abs(q[:, inner] - F * (x[inner] * t + t * t / 2))) <= 1e-13
    assert np.max(np.abs(p[:, inner] - F * x[inner] * t * t / 2)) <= 1e-13


def _forced_wave_error(nr, courant=0.5, T=3.0, w=1.3, k=0.7):
    L = 20.0
    g = _const_grid(nr, 2, -L, L, 0.0, b=1.0)
    n = int(round(T / (courant * g.dr)))
    dt = T / n
    g.dt = dt
    g.set_source(*_profiles(g, lambda x: np.exp(1j * k * x)))
    f = np.array([[np.exp(1j * w * s * dt), np.exp(1j * w * (s + 0.5) * dt)] for s in range(n)])
    z = np.zeros(g.shape, dtype=np.complex128)
    p, q, _ = g.evolve_source(z, z, f)
    x = g.rstar()
    pi_ex = (np.exp(1j * (w * T + k * x)) - np.exp(1j * k * (x + T))) / (1j * (w - k))
    phi_ex = np.exp(1j * k * (x - T)) / (1j * (w - k)) * ((np.exp(1j * (w + k) * T) - 1) / (1j * (w + k))
                                                         - (np.exp(2j * k * T) - 1) / (2j * k))
    sel = np.abs(x) <= 10.0  # far from both radial boundaries (T = 3, speed 1)
    return max(np.max(np.abs(q[0, sel] - pi_ex[sel])), np.max(np.abs(p[0, sel] - phi_ex[sel])))


def test_forced_wave_second_order():
    e = [_forced_wave_error(nr) for nr in (401, 801, 1601)]
    assert e[2] < 1e-3
    for a, b in zip(e, e[1:]):
        assert 3.6 <= a / b <= 4.4, e
