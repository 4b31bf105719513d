"""Pins of the oracle's Lax-Wendroff scheme, Eqs. (lw1)-(lw2) (CPU).

Constant-coefficient cases reduce the system to textbook problems with
closed-form solutions:
* b = 1, everything else 0: d_t Phi + Phi' = Pi, d_t Pi - Pi' = 0, whose
  solution is Phi = Phi0(x - t) + (P(x + t) - P(x - t))/2 with P' = Pi0.
  At Courant number 1 and Pi0 = 0 the two-step scheme translates Phi by
  exactly one cell per step; otherwise it converges at 2nd order.
* A2 = kappa, b = 1, everything else 0, data uniform in r* and equal to
  cos(n th_j) (or sin(n th_j) for the anti-mirror ghosts): the three-point
  theta operator has the exact eigenvalue -(4/dth^2) sin^2(n dth/2), and the
  two stages act as the midpoint rule, so each step multiplies (phi, pi) by
  I + dt S + dt^2 S^2 / 2 with S = [[0, 1], [-w^2, 0]].
* Superposition (complex linearity) of the Kerr step.
"""
import math

import numpy as np
import pytest
from scipy.special import erf

import oracle
from paper_1010_3816_amd import inputs

NC = oracle.NCOEF


def _const_grid(nr, nth, rmin, rmax, dt, m=0, **coef):
    g = oracle.OracleGrid(0.0, 0, m, nr, nth, rmin, rmax, dt, kerr=False)
    ci = np.zeros((NC, nth, nr))
    ch = np.zeros((NC, nth, nr - 1))
    names = oracle.COEF_NAMES
    for k, v in coef.items():
        ci[names.index(k)] = v
        ch[names.index(k)] = v
    g.set_coefficients(ci, ch)
    return g


def test_dalembert_exact_translation_courant_one():
    nr, nth = 200, 2
    g = _const_grid(nr, nth, -10.0, 10.0, 0.0, b=1.0)
    g.dt = g.dr                          # Courant number exactly 1
    x = g.rstar()
    prof = np.exp(-((x + 4.0) ** 2)) * (1 + 0.3j)
    phi = np.tile(prof, (nth, 1))
    pi = np.zeros_like(phi)
    phi, pi = g.project(phi, pi)
    phi0 = phi.copy()
    n = 40
    phi_n, pi_n = g.step(phi, pi, n)
    expect = np.zeros_like(phi0)
    expect[:, n + 1:nr - 1] = phi0[:, 1:nr - 1 - n]
    assert np.max(np.abs(phi_n - expect)) <= 1e-14 * np.max(np.abs(phi0))
    assert np.max(np.abs(pi_n)) == 0.0


def _dalembert_error(nr, courant=0.5, T=4.0):
    L = 20.0
    g = _const_grid(nr, 2, -L, L, 0.0, b=1.0)
    n = int(round(T / (courant * g.dr)))
    g.dt = T / n
    x = g.rstar()
    sig = 1.5

    def phi0(z):
        return np.exp(-((z - 2.0) ** 2) / 2.0)

    def pi0(z):
        return np.exp(-(z**2) / (2 * sig**2))

    def P(z):
        return sig * math.sqrt(math.pi / 2) * erf(z / (sig * math.sqrt(2)))

    phi = np.tile(phi0(x).astype(complex), (2, 1))
    pi = np.tile(pi0(x).astype(complex), (2, 1))
    phi, pi = g.project(phi, pi)
    phi_n, pi_n = g.step(phi, pi, n)
    exact_phi = phi0(x - T) + 0.5 * (P(x + T) - P(x - T))
    exact_pi = pi0(x + T)
    inner = np.abs(x) < 8.0
    return max(np.max(np.abs(phi_n[0, inner] - exact_phi[inner])),
               np.max(np.abs(pi_n[0, inner] - exact_pi[inner])))


def test_dalembert_second_order_convergence():
    e = [_dalembert_error(nr) for nr in (201, 401, 801)]
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert 3.5 < r1 < 4.5 and 3.7 < r2 < 4.3, (e, r1, r2)
    assert e[2] < 5e-3


@pytest.mark.parametrize("m,n", [(0, 1), (2, 3), (1, 2), (3, 5)])
def test_exact_angular_eigenmode(m, n):
    """Uniform-in-r* data on the exact discrete eigenmode of the theta stencil."""
    nr, nth, kappa = 40, 24, 0.37
    dt = 0.05
    g = _const_grid(nr, nth, 0.0, 10.0, dt, m=m, b=1.0, a2=kappa)
    th = g.theta()
    sigma = 1 if m % 2 == 0 else -1
    mode = np.cos(n * th) if sigma == 1 else np.sin(n * th)
    p0, q0 = 0.8 - 0.2j, 0.3 + 0.5j
    phi = np.outer(mode, np.full(nr, p0))
    pi = np.outer(mode, np.full(nr, q0))
    steps = 6
    phi_n, pi_n = g.step(phi, pi, steps)
    w2 = kappa * (4.0 / g.dth**2) * math.sin(n * g.dth / 2) ** 2
    S = np.array([[0.0, 1.0], [-w2, 0.0]])
    G = np.eye(2) + dt * S + 0.5 * dt * dt * S @ S
    pn, qn = np.linalg.matrix_power(G, steps) @ np.array([p0, q0])
    interior = slice(steps + 1, nr - 1 - steps)
    scale = abs(p0) + abs(q0)
    assert np.max(np.abs(phi_n[:, interior] - np.outer(mode, np.full(nr, pn))[:, interior])) < 1e-13 * scale
    assert np.max(np.abs(pi_n[:, interior] - np.outer(mode, np.full(nr, qn))[:, interior])) < 1e-13 * scale
    # the midpoint-rule amplification is slightly above one: |g|^2 = 1 + (w dt)^4 / 4
    lam = np.linalg.eigvals(G)
    assert np.allclose(np.abs(lam) ** 2, 1 + (math.sqrt(w2) * dt) ** 4 / 4, rtol=1e-12)


@pytest.mark.parametrize("a,s,m", [(0.0, -2, 2), (0.7, -2, 1), (0.95, 0, -3)])
def test_superposition(a, s, m):
    nr, nth = 60, 12
    g = oracle.OracleGrid(a, s, m, nr, nth, -20.0, 40.0, 0.01)
    u1 = inputs.random_state(nr, nth, 1)
    u2 = inputs.random_state(nr, nth, 2)
    al, be = 0.3 - 1.1j, -0.7 + 0.4j
    comb = [al * p + be * q for p, q in zip(u1, u2)]
    out1 = g.step(*u1, 3)
    out2 = g.step(*u2, 3)
    outc = g.step(*comb, 3)
    for k in range(2):
        lhs = outc[k]
        rhs = al * out1[k] + be * out2[k]
        assert np.max(np.abs(lhs - rhs)) <= 1e-13 * np.max(np.abs(rhs))
