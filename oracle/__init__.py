"""Teukolsky Lax-Wendroff oracle -- TEST INFRASTRUCTURE ONLY.

ctypes wrapper around ``teuk_oracle.c``: a plain, unfused CPU FP64
implementation of the two-step Lax-Wendroff evolution of the homogeneous
Teukolsky equation (arXiv:1010.3816, Sec. 3, Eqs. (1), (lw1), (lw2) and the
boundary conditions that follow them).  Only ``tests/``, the smoke check and
the benchmark's CPU-baseline leg may import this package; the GPU library
never does, and the two share no code.  The shared library is compiled by
``__graft_entry__.build()`` (gcc, -O2, OpenMP).

Array conventions: complex128 numpy arrays of shape (ntheta, nr), r* fastest.
Coefficient tables have shape (9, ntheta, nr) at integer points and
(9, ntheta, nr-1) at half points, in the order
b, Re c, Im c, Re Ct, Im Ct, A2, A1, Re V0, Im V0.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libteuk_oracle.so")
NCOEF = 9
COEF_NAMES = ("b", "c_re", "c_im", "ct_re", "ct_im", "a2", "a1", "v0_re", "v0_im")

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"oracle library not built: {LIB_PATH} (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    D = ctypes.c_double
    I = ctypes.c_int
    lib.orc_create.restype = P
    lib.orc_create.argtypes = [D, I, I, I, I, D, D, D, I]
    lib.orc_destroy.argtypes = [P]
    lib.orc_set_coefficients.argtypes = [P, P, P]
    lib.orc_get_coefficients.argtypes = [P, P, P, P, P]
    lib.orc_get_x.argtypes = [P, P, P]
    lib.orc_dr.restype = D
    lib.orc_dr.argtypes = [P]
    lib.orc_dth.restype = D
    lib.orc_dth.argtypes = [P]
    lib.orc_set_dt.argtypes = [P, D]
    lib.orc_tortoise_x.restype = I
    lib.orc_tortoise_x.argtypes = [D, D, ctypes.POINTER(D)]
    lib.orc_rstar_of_x.restype = D
    lib.orc_rstar_of_x.argtypes = [D, D]
    lib.orc_coefficients.restype = I
    lib.orc_coefficients.argtypes = [D, I, I, D, D, P, P]
    lib.orc_project.argtypes = [P, P, P]
    lib.orc_extract.argtypes = [P, P, D, D, P]
    lib.orc_step.argtypes = [P, P, P]
    lib.orc_evolve.argtypes = [P, P, P, ctypes.c_int64, I, P, P, P]
    lib.orc_num_threads.restype = I
    lib.orc_set_num_threads.argtypes = [I]
    lib.orc_set_source.argtypes = [P, P, P]
    lib.orc_evolve_source.argtypes = [P, P, P, ctypes.c_int64, P, I, P, P, P]
    lib.orc_mode_sum.restype = I
    lib.orc_mode_sum.argtypes = [D, ctypes.c_int64, I, P, I, P, P, P, P]
    for name, argt in _ADJOINT_SIGS.items():
        fn = getattr(lib, name, None)
        if fn is not None:
            fn.argtypes = argt
            fn.restype = None
    _lib = lib
    return lib


_P = ctypes.c_void_p
_ADJOINT_SIGS = {
    "orc_adjoint_step": [_P, _P, _P],
    "orc_tangent_a": [_P, _P, _P, _P, _P],
    "orc_extract_adjoint": [_P, _P, ctypes.c_double, ctypes.c_double, _P],
    "orc_adjoint_evolve": [_P, _P, _P, ctypes.c_int64, ctypes.c_int, _P, _P, _P, _P, _P, _P],
}


def _ptr(arr):
    return arr.ctypes.data_as(ctypes.c_void_p)


def _c128(arr, shape=None):
    out = np.ascontiguousarray(arr, dtype=np.complex128)
    if shape is not None and out.shape != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {out.shape}")
    return out


def num_threads():
    return _load().orc_num_threads()


def set_num_threads(n):
    """Threads of later oracle calls (timing only: the results do not
    depend on it)."""
    _load().orc_set_num_threads(int(n))


def tortoise_x(a, rstar):
    """x = r - r_+ solving r*(r) = rstar (Kerr, M = 1)."""
    x = ctypes.c_double()
    rc = _load().orc_tortoise_x(float(a), float(rstar), ctypes.byref(x))
    if rc:
        raise ValueError("tortoise inversion failed")
    return x.value


def rstar_of_x(a, x):
    return _load().orc_rstar_of_x(float(a), float(x))


def coefficients(a, s, m, rstar, theta):
    """(values[9], d/da[9]) of the first-order-system coefficients at (r*, theta)."""
    val = np.zeros(NCOEF)
    dval = np.zeros(NCOEF)
    rc = _load().orc_coefficients(float(a), int(s), int(m), float(rstar), float(theta), _ptr(val), _ptr(dval))
    if rc:
        raise ValueError("tortoise inversion failed")
    return val, dval


def mode_sum(a, modes, rstar, phi, samples):
    """Psi at observers (r*_o, phi_o) from mode samples (Sec. 3.2: Psi = sum_m
    e^{i m phi} r^3 Phi_m): samples [n_samples][n_modes][n_obs] -> psi
    [n_samples][n_obs], r from the tortoise inversion for spin a."""
    m = np.ascontiguousarray(modes, dtype=np.int32)
    rs = np.ascontiguousarray(rstar, dtype=np.float64)
    ph = np.ascontiguousarray(phi, dtype=np.float64)
    smp = np.ascontiguousarray(samples, dtype=np.complex128)
    ns, nm, no = smp.shape
    if nm != m.size or no != rs.size or no != ph.size:
        raise ValueError("samples must have shape (n_samples, len(modes), len(observers))")
    psi = np.zeros((ns, no), dtype=np.complex128)
    if _load().orc_mode_sum(float(a), ns, nm, _ptr(m), no, _ptr(rs), _ptr(ph), _ptr(smp), _ptr(psi)):
        raise ValueError("tortoise inversion failed")
    return psi


class OracleGrid:
    """One (r*, theta) grid for one (a, s, m); kerr=False expects user tables."""

    def __init__(self, a, s, m, nr, ntheta, rstar_min, rstar_max, dt, kerr=True):
        self._lib = _load()
        self.a, self.s, self.m = float(a), int(s), int(m)
        self.nr, self.ntheta = int(nr), int(ntheta)
        self.rstar_min, self.rstar_max = float(rstar_min), float(rstar_max)
        self._h = self._lib.orc_create(self.a, self.s, self.m, self.nr, self.ntheta,
                                       self.rstar_min, self.rstar_max, float(dt), 1 if kerr else 0)
        if not self._h:
            raise ValueError("invalid oracle grid parameters")
        self.dr = self._lib.orc_dr(self._h)
        self.dth = self._lib.orc_dth(self._h)
        self._dt = float(dt)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_destroy(h)
            self._h = None

    @property
    def dt(self):
        return self._dt

    @dt.setter
    def dt(self, v):
        self._dt = float(v)
        self._lib.orc_set_dt(self._h, self._dt)

    @property
    def shape(self):
        return (self.ntheta, self.nr)

    def rstar(self):
        return self.rstar_min + np.arange(self.nr) * self.dr

    def rstar_half(self):
        return self.rstar_min + (np.arange(self.nr - 1) + 0.5) * self.dr

    def theta(self):
        return (np.arange(self.ntheta) + 0.5) * self.dth

    def set_coefficients(self, ci, ch):
        ci = np.ascontiguousarray(ci, dtype=np.float64).reshape(NCOEF, self.ntheta, self.nr)
        ch = np.ascontiguousarray(ch, dtype=np.float64).reshape(NCOEF, self.ntheta, self.nr - 1)
        self._lib.orc_set_coefficients(self._h, _ptr(ci), _ptr(ch))

    def coefficients(self):
        ci = np.zeros((NCOEF, self.ntheta, self.nr))
        ch = np.zeros((NCOEF, self.ntheta, self.nr - 1))
        dci = np.zeros_like(ci)
        dch = np.zeros_like(ch)
        self._lib.orc_get_coefficients(self._h, _ptr(ci), _ptr(ch), _ptr(dci), _ptr(dch))
        return ci, ch, dci, dch

    def x_tables(self):
        xi = np.zeros(self.nr)
        xh = np.zeros(self.nr - 1)
        self._lib.orc_get_x(self._h, _ptr(xi), _ptr(xh))
        return xi, xh

    def project(self, phi, pi):
        """Copy with Phi = Pi = 0 on the radial boundary columns."""
        phi = _c128(phi, self.shape).copy()
        pi = _c128(pi, self.shape).copy()
        self._lib.orc_project(self._h, _ptr(phi), _ptr(pi))
        return phi, pi

    def step(self, phi, pi, n=1):
        phi = _c128(phi, self.shape).copy()
        pi = _c128(pi, self.shape).copy()
        if n == 1:
            self._lib.orc_step(self._h, _ptr(phi), _ptr(pi))
        else:
            self._lib.orc_evolve(self._h, _ptr(phi), _ptr(pi), int(n), 0, None, None, None)
        return phi, pi

    def evolve(self, phi, pi, n, ext_rstar=(), ext_theta=()):
        """n steps; returns (phi, pi, series[n, n_ext]) with Phi sampled after each step."""
        phi = _c128(phi, self.shape).copy()
        pi = _c128(pi, self.shape).copy()
        er = np.ascontiguousarray(ext_rstar, dtype=np.float64).ravel()
        et = np.ascontiguousarray(ext_theta, dtype=np.float64).ravel()
        if er.shape != et.shape:
            raise ValueError("extraction coordinate arrays differ in length")
        ne = er.size
        series = np.zeros((int(n), ne), dtype=np.complex128)
        self._lib.orc_evolve(self._h, _ptr(phi), _ptr(pi), int(n), ne,
                             _ptr(er) if ne else None, _ptr(et) if ne else None,
                             _ptr(series) if ne else None)
        return phi, pi, series

    def set_source(self, gi, gh):
        """Source profile g of the inhomogeneous variant at integer (ntheta, nr)
        and half (ntheta, nr-1) positions; None removes it."""
        if gi is None or gh is None:
            self._lib.orc_set_source(self._h, None, None)
            return
        gi = _c128(gi, self.shape)
        gh = _c128(gh, (self.shape[0], self.shape[1] - 1))
        self._lib.orc_set_source(self._h, _ptr(gi), _ptr(gh))

    def evolve_source(self, phi, pi, f, ext_rstar=(), ext_theta=()):
        """n = len(f) steps of the inhomogeneous variant; f[k] = (f(t_k),
        f(t_k + dt/2)) for step k.  Returns (phi, pi, series[n, n_ext])."""
        phi = _c128(phi, self.shape).copy()
        pi = _c128(pi, self.shape).copy()
        f = np.ascontiguousarray(f, dtype=np.complex128)
        n = f.shape[0]
        if f.shape != (n, 2):
            raise ValueError("f must have shape (n, 2)")
        er = np.ascontiguousarray(ext_rstar, dtype=np.float64).ravel()
        et = np.ascontiguousarray(ext_theta, dtype=np.float64).ravel()
        ne = er.size
        series = np.zeros((n, ne), dtype=np.complex128)
        self._lib.orc_evolve_source(self._h, _ptr(phi), _ptr(pi), n, _ptr(f), ne,
                                    _ptr(er) if ne else None, _ptr(et) if ne else None,
                                    _ptr(series) if ne else None)
        return phi, pi, series

    def extract(self, phi, rstar, theta):
        phi = _c128(phi, self.shape)
        out = np.zeros(1, dtype=np.complex128)
        self._lib.orc_extract(self._h, _ptr(phi), float(rstar), float(theta), _ptr(out))
        return complex(out[0])

    # ---- adjoint -----------------------------------------------------------
    def adjoint_step(self, lam_phi, lam_pi):
        """A^H applied to the cotangent of the state after one step."""
        lp = _c128(lam_phi, self.shape).copy()
        lq = _c128(lam_pi, self.shape).copy()
        self._lib.orc_adjoint_step(self._h, _ptr(lp), _ptr(lq))
        return lp, lq

    def tangent_a(self, phi, pi):
        """(dA/da) u: derivative of one step with respect to the spin at fixed u."""
        phi = _c128(phi, self.shape)
        pi = _c128(pi, self.shape)
        tp = np.zeros(self.shape, dtype=np.complex128)
        tq = np.zeros(self.shape, dtype=np.complex128)
        self._lib.orc_tangent_a(self._h, _ptr(phi), _ptr(pi), _ptr(tp), _ptr(tq))
        return tp, tq

    def evolve_spin_tangent(self, phi, pi, vphi, vpi, n, ext_rstar=(), ext_theta=()):
        """n steps of the state u and of its spin derivative v = du/da by the
        tangent-linear step of Eqs. (lw1)-(lw2): v <- A v + (dA/da) u, with u
        the state before the step, then u <- A u.  Returns
        (phi, pi, vphi, vpi, series, tseries): the samples of Phi and of its
        a-derivative after each step, shape (n, n_ext).  A composition of
        step, tangent_a and extract, step by step."""
        p, q = _c128(phi, self.shape).copy(), _c128(pi, self.shape).copy()
        vp, vq = _c128(vphi, self.shape).copy(), _c128(vpi, self.shape).copy()
        er = np.ascontiguousarray(ext_rstar, dtype=np.float64).ravel()
        et = np.ascontiguousarray(ext_theta, dtype=np.float64).ravel()
        series = np.zeros((int(n), er.size), dtype=np.complex128)
        tseries = np.zeros_like(series)
        for k in range(int(n)):
            tp, tq = self.tangent_a(p, q)
            vp, vq = self.step(vp, vq, 1)
            vp, vq = vp + tp, vq + tq
            p, q = self.step(p, q, 1)
            for e in range(er.size):
                series[k, e] = self.extract(p, er[e], et[e])
                tseries[k, e] = self.extract(vp, er[e], et[e])
        return p, q, vp, vq, series, tseries

    def extract_adjoint(self, lam_phi, rstar, theta, gval):
        lp = _c128(lam_phi, self.shape).copy()
        g = np.array([gval], dtype=np.complex128)
        self._lib.orc_extract_adjoint(self._h, _ptr(lp), float(rstar), float(theta), _ptr(g))
        return lp

    def adjoint_evolve(self, phi0, pi0, n, ext_rstar, ext_theta, grad_series):
        """Reverse pass of n steps: (dL/dphi0, dL/dpi0, dL/da) for a loss with
        gradient grad_series (n x n_ext, PyTorch complex convention) with
        respect to the extraction series of evolve()."""
        phi0 = _c128(phi0, self.shape)
        pi0 = _c128(pi0, self.shape)
        er = np.ascontiguousarray(ext_rstar, dtype=np.float64).ravel()
        et = np.ascontiguousarray(ext_theta, dtype=np.float64).ravel()
        gs = np.ascontiguousarray(grad_series, dtype=np.complex128).reshape(int(n), er.size)
        lp = np.zeros(self.shape, dtype=np.complex128)
        lq = np.zeros(self.shape, dtype=np.complex128)
        out = ctypes.c_double()
        self._lib.orc_adjoint_evolve(self._h, _ptr(phi0), _ptr(pi0), int(n), int(er.size), _ptr(er), _ptr(et),
                                     _ptr(gs), _ptr(lp), _ptr(lq), ctypes.byref(out))
        return lp, lq, out.value
