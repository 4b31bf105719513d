"""Seeded synthetic inputs for the Teukolsky Lax-Wendroff evolution.

This module is shared by the tests of the GPU library and of the CPU oracle.
It holds no arithmetic of the method itself: only the grid placement needed
to sample initial data, the initial pulses, the seeded parameter draws of the
standard workloads, and the run-parameter recipe for the time step.

Workloads (the paper sizes its grids to fill device memory and gives no
grid sizes, Sec. 4; these are synthetic stand-ins):

* ``schwarzschild_400x32``: a=0, s=-2, m=2, 400 x 32, r* in [-50, 150],
  Phi0 = exp(-(r*-10)^2/(2*4^2)) (1 - cos th)^2, Pi0 = 0, 1000 steps,
  extraction at (r* = 100, th = pi/2).
* ``kerr_a0.9_6400x256``: a=0.9, s=-2, m=2, 6400 x 256, r* in [-100, 600],
  rng(1010): centre ~ U[5, 20], then width ~ U[2, 6]; regular angular
  profile; 20000 steps; extraction at (500, pi/2).
* ``kerr_a0.99_25600x512``: a=0.99, s=-2, m=2, 25600 x 512,
  r* in [-200, 1200], rng(1011), 10000 steps.
* ``batch64``: 64 members drawn from rng(1012) in the order
  nr ~ U{1600..12800}, ntheta ~ {64, 128, 256}, m ~ U{-4..4}, s ~ {0, -2},
  a ~ U[0, 0.99], centre ~ U[5, 20], width ~ U[2, 6]; r* in [-100, 600];
  5000 steps each.
* ``adjoint_a0.7_6400x256``: a=0.7, s=-2, m=2, 6400 x 256, r* in
  [-100, 600], rng(1013) pulse, 8000 steps, checkpoint every 100 steps.
  At the stable time step the run covers t ~ 11.7 M, so a signal from the
  pulse (centre ~ 17 M) cannot reach r* = 500 M: the extraction point is
  moved inside the light cone, to r* = 25 M (about centre + t/2), theta =
  pi/2.  The loss target is the series of a perturbed run (a + 0.01, centre
  + 0.5), see ``adjoint_target``.
"""
import math

import numpy as np

# ---------------------------------------------------------------------------
# grid placement (r* endpoints on the grid, cell-centred theta)
# ---------------------------------------------------------------------------


def rstar_grid(nr, rstar_min, rstar_max):
    dr = (rstar_max - rstar_min) / (nr - 1)
    return rstar_min + np.arange(nr) * dr


def theta_grid(ntheta):
    return (np.arange(ntheta) + 0.5) * (math.pi / ntheta)


def regular_profile(theta, m, s):
    """sin^|m+s|(th/2) cos^|m-s|(th/2): vanishes at each pole as the angular
    potential (m + s cos th)^2 / sin^2 th requires."""
    return np.sin(theta / 2) ** abs(m + s) * np.cos(theta / 2) ** abs(m - s)


def gaussian_pulse(nr, ntheta, rstar_min, rstar_max, center, width, profile="regular", m=2, s=-2):
    """(phi0, pi0) complex128 arrays of shape (ntheta, nr):
    Phi0 = exp(-(r* - center)^2 / (2 width^2)) * S(theta), Pi0 = 0.

    profile: "regular" (see regular_profile), "one_minus_cos_sq" ((1 - cos th)^2),
    "one_plus_cos_sq" ((1 + cos th)^2) or a callable of theta."""
    rs = rstar_grid(nr, rstar_min, rstar_max)
    th = theta_grid(ntheta)
    if callable(profile):
        ang = profile(th)
    elif profile == "regular":
        ang = regular_profile(th, m, s)
    elif profile == "one_minus_cos_sq":
        ang = (1.0 - np.cos(th)) ** 2
    elif profile == "one_plus_cos_sq":
        ang = (1.0 + np.cos(th)) ** 2
    else:
        raise ValueError(f"unknown profile {profile!r}")
    radial = np.exp(-((rs - center) ** 2) / (2.0 * width * width))
    phi0 = (ang[:, None] * radial[None, :]).astype(np.complex128)
    pi0 = np.zeros_like(phi0)
    return phi0, pi0


def random_state(nr, ntheta, seed):
    """Dense seeded complex data (for linearity / adjoint identities)."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((2, ntheta, nr)) + 1j * rng.standard_normal((2, ntheta, nr))
    return a[0].astype(np.complex128), a[1].astype(np.complex128)


# ---------------------------------------------------------------------------
# run-parameter recipe for the time step
# ---------------------------------------------------------------------------

# Upper bound of Delta / Sigma^2 over r > r_+, all theta, 0 <= a <= 0.99
# (it peaks near r = 2.5-3 M at about 0.045 for a = 0.99 and 1/27 for a = 0).
_A2_BOUND = 0.05


def angular_frequency_bound(ntheta, m, s):
    """Crude bound of the largest angular frequency on the grid: the
    three-point theta operator contributes at most 4/dth^2 and the pole
    potential (m + s cos th)^2 / sin^2 th is largest on the rows nearest the
    poles; both are weighted by the bound of Delta/Sigma^2."""
    dth = math.pi / ntheta
    th = theta_grid(ntheta)
    pole = np.max((m + s * np.cos(th)) ** 2 / np.sin(th) ** 2) + abs(s)
    return math.sqrt(_A2_BOUND * (4.0 / dth**2 + pole))


def stable_dt(dr, ntheta, m, s, n_steps, growth=10.0, courant=0.5):
    """Time step used by the workloads: min(courant * dr, dt_growth) where
    dt_growth bounds the amplification of the fastest angular mode over
    n_steps steps to `growth`.  For modes smooth in r* the two stages act as
    the midpoint rule, whose amplification g = 1 + z + z^2/2 (z = i w dt)
    has |g|^2 = 1 + (w dt)^4 / 4, so n steps grow by exp(n (w dt)^4 / 8)."""
    w = angular_frequency_bound(ntheta, m, s)
    dt_g = (8.0 * math.log(growth) / max(int(n_steps), 1)) ** 0.25 / w
    return min(courant * dr, dt_g)


# ---------------------------------------------------------------------------
# standard workloads
# ---------------------------------------------------------------------------


def _pulse_draw(seed):
    rng = np.random.default_rng(seed)
    center = rng.uniform(5.0, 20.0)
    width = rng.uniform(2.0, 6.0)
    return float(center), float(width)


def workload(name):
    """Parameter dict of a standard workload (no arrays)."""
    if name == "schwarzschild_400x32":
        w = dict(a=0.0, s=-2, m=2, nr=400, ntheta=32, rstar_min=-50.0, rstar_max=150.0,
                 center=10.0, width=4.0, profile="one_minus_cos_sq", steps=1000,
                 extract_rstar=[100.0], extract_theta=[math.pi / 2])
    elif name == "kerr_a0.9_6400x256":
        c, wd = _pulse_draw(1010)
        w = dict(a=0.9, s=-2, m=2, nr=6400, ntheta=256, rstar_min=-100.0, rstar_max=600.0,
                 center=c, width=wd, profile="regular", steps=20000,
                 extract_rstar=[500.0], extract_theta=[math.pi / 2])
    elif name == "kerr_a0.99_25600x512":
        c, wd = _pulse_draw(1011)
        w = dict(a=0.99, s=-2, m=2, nr=25600, ntheta=512, rstar_min=-200.0, rstar_max=1200.0,
                 center=c, width=wd, profile="regular", steps=10000,
                 extract_rstar=[], extract_theta=[])
    elif name == "adjoint_a0.7_6400x256":
        c, wd = _pulse_draw(1013)
        w = dict(a=0.7, s=-2, m=2, nr=6400, ntheta=256, rstar_min=-100.0, rstar_max=600.0,
                 center=c, width=wd, profile="regular", steps=8000, checkpoint_every=100,
                 extract_rstar=[25.0], extract_theta=[math.pi / 2])
    else:
        raise KeyError(name)
    w["name"] = name
    w["dr"] = (w["rstar_max"] - w["rstar_min"]) / (w["nr"] - 1)
    w["dt_literal"] = 0.5 * w["dr"]
    w["dt"] = stable_dt(w["dr"], w["ntheta"], w["m"], w["s"], w["steps"])
    return w


def adjoint_target(w):
    """Parameters of the perturbed run whose extraction series is the loss
    target of the adjoint workload: spin + 0.01 and pulse centre + 0.5 M,
    everything else (grid, time step, width, extraction point) unchanged."""
    t = dict(w)
    t["a"] = w["a"] + 0.01
    t["center"] = w["center"] + 0.5
    return t


def batch_members(seed=1012, count=64, rstar_min=-100.0, rstar_max=600.0, steps=5000):
    """The batched workload's members, drawn in a fixed order from one rng."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        nr = int(rng.integers(1600, 12801))
        ntheta = int(rng.choice([64, 128, 256]))
        m = int(rng.integers(-4, 5))
        s = int(rng.choice([0, -2]))
        a = float(rng.uniform(0.0, 0.99))
        center = float(rng.uniform(5.0, 20.0))
        width = float(rng.uniform(2.0, 6.0))
        dr = (rstar_max - rstar_min) / (nr - 1)
        out.append(dict(index=k, a=a, s=s, m=m, nr=nr, ntheta=ntheta, rstar_min=rstar_min,
                        rstar_max=rstar_max, center=center, width=width, profile="regular",
                        steps=steps, dr=dr, dt=stable_dt(dr, ntheta, m, s, steps)))
    return out


def initial_data(w, profile=None):
    """(phi0, pi0) for a workload dict."""
    return gaussian_pulse(w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["center"], w["width"],
                          profile or w["profile"], w["m"], w["s"])


# ---------------------------------------------------------------------------
# a source for the inhomogeneous variant (the paper gives no source model)
# ---------------------------------------------------------------------------


def localised_source(nr, ntheta, rstar_min, rstar_max, center, width=1.0, theta0=math.pi / 2, theta_width=0.1):
    """(gi, gh) complex128 profiles of a separable source f(t) g(r*, theta):
    g = exp(-(r* - center)^2 / (2 width^2)) exp(-(theta - theta0)^2 / (2
    theta_width^2)), a blob standing in for a particle's neighbourhood,
    sampled at the grid columns (gi, shape (ntheta, nr)) and at the half
    positions between them (gh, shape (ntheta, nr - 1))."""
    x = rstar_grid(nr, rstar_min, rstar_max)
    xh = 0.5 * (x[1:] + x[:-1])
    ang = np.exp(-((theta_grid(ntheta) - theta0) ** 2) / (2.0 * theta_width**2))[:, None]
    gi = ang * np.exp(-((x - center) ** 2) / (2.0 * width**2))[None, :] + 0j
    gh = ang * np.exp(-((xh - center) ** 2) / (2.0 * width**2))[None, :] + 0j
    return gi, gh


def oscillating_factors(n, dt, omega=0.4, amplitude=50.0, t0=0.0):
    """Time factors of n steps for teuk_step_n_source: row k holds
    (f(t_k), f(t_k + dt/2)) with f(t) = amplitude exp(i omega t), t_k = t0 + k dt."""
    t = t0 + np.arange(n) * dt
    return amplitude * np.stack([np.exp(1j * omega * t), np.exp(1j * omega * (t + 0.5 * dt))], axis=1)
