"""Pins of the oracle's field-from-modes sum (Sec. 3.2: Psi = sum over m of
exp(i m phi) r^3 Phi_m) to things other than its own formula:

 * a discrete Fourier transform (numpy's FFT) over equally spaced azimuths
   recovers r^3 Phi_m in the bin of m, and nothing elsewhere: fixes the sign
   of the exponent, the radial factor and the order of the modes;
 * a single m = 0 mode of unit amplitude at r* = 4 in Schwarzschild, where
   r* = r + 2 ln(r/2 - 1) gives r = 4 exactly: Psi = 64;
 * linearity in the samples.
"""
import math

import numpy as np

import oracle


def test_dft_over_azimuth_recovers_each_mode():
    a, rs, N = 0.7, 37.5, 16
    modes = [-3, -1, 0, 2, 3, 5]
    rng = np.random.default_rng(1)
    S = rng.standard_normal((4, len(modes))) + 1j * rng.standard_normal((4, len(modes)))
    phi = 2 * math.pi * np.arange(N) / N
    samples = np.repeat(S[:, :, None], N, axis=2)  # the modes do not depend on the azimuth
    psi = oracle.mode_sum(a, modes, [rs] * N, phi, samples)
    r3 = (1 + math.sqrt(1 - a * a) + oracle.tortoise_x(a, rs)) ** 3
    F = np.fft.fft(psi, axis=1) / N
    bins = {m % N: j for j, m in enumerate(modes)}
    for q in range(N):
        want = r3 * S[:, bins[q]] if q in bins else np.zeros(4)
        assert np.max(np.abs(F[:, q] - want)) <= 1e-13 * r3 * np.max(np.abs(S)), q


def test_single_axisymmetric_mode_schwarzschild():
    psi = oracle.mode_sum(0.0, [0], [4.0], [1.234], np.ones((1, 1, 1), dtype=np.complex128))
    assert abs(psi[0, 0] - 64.0) <= 1e-12 * 64.0


def test_linear_in_samples():
    rng = np.random.default_rng(2)
    modes, rs, ph = [-2, 0, 1], [10.0, 50.0], [0.3, -2.0]
    A = rng.standard_normal((3, 3, 2)) + 1j * rng.standard_normal((3, 3, 2))
    B = rng.standard_normal((3, 3, 2)) + 1j * rng.standard_normal((3, 3, 2))
    c = 0.7 - 1.3j
    lhs = oracle.mode_sum(0.5, modes, rs, ph, A + c * B)
    rhs = oracle.mode_sum(0.5, modes, rs, ph, A) + c * oracle.mode_sum(0.5, modes, rs, ph, B)
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * np.max(np.abs(lhs))
