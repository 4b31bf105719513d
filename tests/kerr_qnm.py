"""Kerr quasinormal frequencies by Leaver's continued-fraction method
(E. W. Leaver, Proc. R. Soc. Lond. A 402 (1985) 285) -- test infrastructure.

An independent physics reference for the oracle's Kerr evolution: it shares
nothing with the oracle (no coefficient tables, no tortoise coordinate, no
time stepping).  The perturbation exp(-i w t + i m phi) S(theta) R(r) of
spin weight s separates; both the angular and the radial function are
expanded in series whose coefficients obey three-term recurrences, and a
solution that is regular (angular) or has quasinormal boundary behaviour
(radial) exists exactly when the corresponding continued fraction
vanishes.  The angular fraction fixes the separation constant A(c) for
c = a w; the radial fraction, with that A, fixes w.

Leaver works in units with 2M = 1; the functions here take and return
quantities in units of M (a in [0, 1), M w).
"""
import numpy as np


def _continued_fraction(alpha, beta, gamma):
    """beta_0 - alpha_0 gamma_1 / (beta_1 - alpha_1 gamma_2 / (beta_2 - ...)),
    truncated at the length of the coefficient arrays, evaluated from the
    tail."""
    f = beta[-1]
    for n in range(len(beta) - 2, -1, -1):
        f = beta[n] - alpha[n] * gamma[n + 1] / f
    return f


def angular_fraction(A, c, s, m, depth=60):
    """Angular recurrence of the spin-weighted spheroidal function with
    oblateness c = a w and separation constant A."""
    k1, k2 = abs(m - s) / 2.0, abs(m + s) / 2.0
    n = np.arange(depth, dtype=float)
    alpha = -2.0 * (n + 1) * (n + 2 * k1 + 1)
    beta = (n * (n - 1) + 2 * n * (k1 + k2 + 1 - 2 * c)
            - (2 * c * (2 * k1 + s + 1) - (k1 + k2) * (k1 + k2 + 1))
            - (c * c + s * (s + 1) + A))
    gamma = 2 * c * (n + k1 + k2 + s)
    return _continued_fraction(alpha, beta, gamma)


def _secant(f, x0, x1, tol=1e-12, maxit=100):
    f0, f1 = f(x0), f(x1)
    for _ in range(maxit):
        if f1 == f0:
            break
        x2 = x1 - f1 * (x1 - x0) / (f1 - f0)
        x0, f0 = x1, f1
        x1, f1 = x2, f(x2)
        if abs(x1 - x0) < tol * max(1.0, abs(x1)):
            return x1
    raise RuntimeError("secant iteration did not converge")


def separation_constant(c, s, m, l):
    """A_lm(c), followed from its c = 0 value l(l+1) - s(s+1) (the angular
    equation's spherical limit) in small steps of c.  The plain continued
    fraction used here has, at c = 0, only the root of the lowest multipole
    l = max(|m|, |s|); higher l would need Leaver's inverted fractions."""
    if l != max(abs(m), abs(s)):
        raise ValueError("only the lowest multipole l = max(|m|, |s|) is supported")
    A = complex(l * (l + 1) - s * (s + 1))
    steps = max(1, int(np.ceil(abs(c) / 0.05)))
    for k in range(1, steps + 1):
        ck = c * k / steps
        A = _secant(lambda x: angular_fraction(x, ck, s, m), A, A + 1e-3)
    return A


def radial_fraction(w, a, s, m, A, depth=400):
    """Leaver's radial recurrence (2M = 1 units: 0 <= a < 1/2, w = 2 M omega)
    for the separation constant A."""
    b = np.sqrt(1.0 - 4.0 * a * a)
    q = (w / 2.0 - a * m) / b
    c0 = 1 - s - 1j * w - 2j * q
    c1 = -4 + 2j * w * (2 + b) + 4j * q
    c2 = s + 3 - 3j * w - 2j * q
    c3 = (w * w * (4 + 2 * b - a * a) - 2 * a * m * w - s - 1 + (2 + b) * 1j * w - A
          + (4 * w + 2j) * q)
    c4 = s + 1 - 2 * w * w - (2 * s + 3) * 1j * w - (4 * w + 2j) * q
    n = np.arange(depth, dtype=float)
    alpha = n * n + (c0 + 1) * n + c0
    beta = -2 * n * n + (c1 + 2) * n + c3
    gamma = n * n + (c2 - 3) * n + c4 - c2 + 2
    return _continued_fraction(alpha, beta, gamma)


def kerr_qnm(a, s, m, l, guess):
    """Fundamental quasinormal frequency M omega of spin a (units of M) near
    `guess` (units of 1/M), with the separation constant solved alongside."""
    aL = a / 2.0

    def f(wL):
        A = separation_constant(aL * wL, s, m, l)
        return radial_fraction(wL, aL, s, m, A)

    wL = _secant(f, 2.0 * guess, 2.0 * guess * (1 + 1e-3))
    return wL / 2.0


def kerr_qnm_from_schwarzschild(a, s, m, l, w_schw, step=0.1):
    """The mode followed in spin from its Schwarzschild value w_schw (units of
    1/M) to spin a, in steps of at most `step`."""
    w = kerr_qnm(0.0, s, m, l, w_schw)
    k = max(1, int(np.ceil(a / step)))
    for j in range(1, k + 1):
        w = kerr_qnm(a * j / k, s, m, l, w)
    return w
