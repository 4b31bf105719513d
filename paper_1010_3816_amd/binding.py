"""ctypes binding of libteuk.so (C ABI in include/teuk.h).

The functions below carry the names of the C entry points and only marshal
arguments; every step of the evolution runs in the library's gfx950 kernels.
PyTorch supplies device memory (the workspace and the field tensors) and the
HIP stream.  If the library has not been built this module raises at import:
there is no CPU fallback.
"""
import ctypes

import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# TEUK_LIBRARY may point at another build of the same sources (tuning runs).
LIB_PATH = os.environ.get("TEUK_LIBRARY", os.path.join(_PKG, "libteuk.so"))

TEUK_OK = 0
TEUK_E_INVALID_ARG = -1
TEUK_E_HIP = -2
TEUK_E_NONFINITE = -3
TEUK_E_WORKSPACE = -4
TEUK_E_STATE = -5
TEUK_E_UNSTABLE_DT = -6
TEUK_COEF_KERR = 0
TEUK_COEF_USER = 1
TEUK_NCOEF = 9
TEUK_ADJ_PROJECT_INITIAL = 1
TEUK_ADJ_TANGENT_WINDOW = 2

_ERRNAMES = {-1: "TEUK_E_INVALID_ARG", -2: "TEUK_E_HIP", -3: "TEUK_E_NONFINITE",
             -4: "TEUK_E_WORKSPACE", -5: "TEUK_E_STATE", -6: "TEUK_E_UNSTABLE_DT"}


class TeukError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class teuk_params(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("s", ctypes.c_int32), ("m", ctypes.c_int32),
                ("nr", ctypes.c_int64), ("ntheta", ctypes.c_int64),
                ("rstar_min", ctypes.c_double), ("rstar_max", ctypes.c_double),
                ("dt", ctypes.c_double), ("coef_mode", ctypes.c_int32), ("n_extract", ctypes.c_int32),
                ("extract_rstar", ctypes.POINTER(ctypes.c_double)),
                ("extract_theta", ctypes.POINTER(ctypes.c_double)),
                ("stable_steps", ctypes.c_int64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P, V = ctypes.POINTER(teuk_params), ctypes.c_void_p
    I32, I64, D = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "teuk_workspace_bytes": (ctypes.c_size_t, [P]),
        "teuk_init_grid": (ctypes.c_int, [P, V, V, ctypes.c_size_t, ctypes.POINTER(V)]),
        "teuk_set_coefficients": (ctypes.c_int, [V, V, V]),
        "teuk_set_initial_data": (ctypes.c_int, [V, V, V]),
        "teuk_step_n": (ctypes.c_int, [V, I64, V]),
        "teuk_extract": (ctypes.c_int, [V, I32, V, V, V]),
        "teuk_extract_noalloc": (ctypes.c_int, [V, I32, V, V, V]),
        "teuk_get_state": (ctypes.c_int, [V, V, V]),
        "teuk_check_finite": (ctypes.c_int, [V]),
        "teuk_steps_taken": (I64, [V]),
        "teuk_get_dt": (D, [V]),
        "teuk_set_tile": (ctypes.c_int, [V, I32, I32]),
        "teuk_get_tile": (ctypes.c_int, [V, ctypes.POINTER(I32), ctypes.POINTER(I32)]),
        "teuk_set_steps_per_pass": (ctypes.c_int, [V, I32]),
        "teuk_get_steps_per_pass": (ctypes.c_int, [V, ctypes.POINTER(I32)]),
        "teuk_set_block_launch": (ctypes.c_int, [V, I32, I32]),
        "teuk_get_block_launch": (ctypes.c_int, [V, ctypes.POINTER(I32), ctypes.POINTER(I32)]),
        "teuk_set_cache_policy": (ctypes.c_int, [V, I32]),
        "teuk_spin_tangent_workspace_bytes": (ctypes.c_size_t, [V]),
        "teuk_enable_spin_tangent": (ctypes.c_int, [V, V, ctypes.c_size_t]),
        "teuk_set_spin_tangent": (ctypes.c_int, [V, V, V]),
        "teuk_get_spin_tangent": (ctypes.c_int, [V, V, V]),
        "teuk_step_n_spin_tangent": (ctypes.c_int, [V, I64, V, V]),
        "teuk_spin_gradient": (ctypes.c_int, [V, I64, V, V, V]),
        "teuk_get_cache_policy": (ctypes.c_int, [V, ctypes.POINTER(I32), ctypes.POINTER(I32)]),
        "teuk_set_finite_check": (ctypes.c_int, [V, I64]),
        "teuk_set_adjoint_tile": (ctypes.c_int, [V, I32, I32]),
        "teuk_get_adjoint_tile": (ctypes.c_int, [V, ctypes.POINTER(I32), ctypes.POINTER(I32)]),
        "teuk_suggest_dt": (ctypes.c_int, [P, I64, D, D, ctypes.POINTER(D)]),
        "teuk_free": (ctypes.c_int, [V]),
        "teuk_last_error": (ctypes.c_char_p, []),
        "teuk_window_bytes": (ctypes.c_size_t, [V, I64]),
        "teuk_step_n_store": (ctypes.c_int, [V, I64, V, V]),
        "teuk_step_n_tangent": (ctypes.c_int, [V, I64, V]),
        "teuk_get_window_slot": (ctypes.c_int, [V, V, I64, V, V]),
        "teuk_source_workspace_bytes": (ctypes.c_size_t, [V]),
        "teuk_set_source": (ctypes.c_int, [V, V, ctypes.c_size_t, V, V]),
        "teuk_step_n_source": (ctypes.c_int, [V, I64, V, V]),
        "teuk_adjoint_workspace_bytes": (ctypes.c_size_t, [V]),
        "teuk_enable_adjoint": (ctypes.c_int, [V, V, ctypes.c_size_t]),
        "teuk_adjoint_step_n": (ctypes.c_int, [V, I64, V, V, V, V, I32, ctypes.POINTER(D)]),
        "teuk_adjoint_step_n_async": (ctypes.c_int, [V, I64, V, V, V, V, I32, V]),
        "teuk_batch_workspace_bytes": (ctypes.c_size_t, [P, I32]),
        "teuk_batch_init": (ctypes.c_int, [P, I32, V, V, ctypes.c_size_t, ctypes.POINTER(V)]),
        "teuk_batch_set_initial_data": (ctypes.c_int, [V, I32, V, V]),
        "teuk_batch_get_state": (ctypes.c_int, [V, I32, V, V]),
        "teuk_batch_step_n": (ctypes.c_int, [V, I64]),
        "teuk_batch_set_launch": (ctypes.c_int, [V, I32, I32, I32]),
        "teuk_batch_set_steps_per_pass": (ctypes.c_int, [V, I32]),
        "teuk_batch_extract": (ctypes.c_int, [V, V]),
        "teuk_batch_n_extract": (I32, [V]),
        "teuk_radius": (ctypes.c_int, [D, D, ctypes.POINTER(D)]),
        "teuk_assemble_modes": (ctypes.c_int, [I64, I32, ctypes.POINTER(I32), I32, ctypes.POINTER(D),
                                               ctypes.POINTER(D), V, V, V]),
        "teuk_batch_get_launch": (ctypes.c_int, [V, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32)]),
        "teuk_batch_total_points": (I64, [V]),
        "teuk_batch_free": (ctypes.c_int, [V]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()
EXPORTED = ("teuk_workspace_bytes", "teuk_init_grid", "teuk_set_coefficients", "teuk_set_initial_data",
            "teuk_step_n", "teuk_extract", "teuk_get_state", "teuk_check_finite", "teuk_steps_taken",
            "teuk_get_dt", "teuk_set_tile", "teuk_get_tile", "teuk_suggest_dt", "teuk_free",
            "teuk_last_error", "teuk_window_bytes", "teuk_step_n_store", "teuk_adjoint_workspace_bytes",
            "teuk_enable_adjoint", "teuk_adjoint_step_n", "teuk_set_adjoint_tile", "teuk_get_adjoint_tile",
            "teuk_set_steps_per_pass", "teuk_get_steps_per_pass", "teuk_set_block_launch", "teuk_get_block_launch",
            "teuk_set_cache_policy", "teuk_get_cache_policy",
            "teuk_batch_workspace_bytes", "teuk_batch_init",
            "teuk_batch_set_initial_data", "teuk_batch_get_state", "teuk_batch_step_n", "teuk_batch_set_launch",
            "teuk_batch_get_launch", "teuk_batch_total_points", "teuk_batch_free",
            "teuk_batch_set_steps_per_pass", "teuk_batch_extract", "teuk_batch_n_extract", "teuk_radius",
            "teuk_assemble_modes", "teuk_set_finite_check", "teuk_extract_noalloc",
            "teuk_step_n_tangent", "teuk_get_window_slot", "teuk_source_workspace_bytes", "teuk_set_source",
            "teuk_step_n_source", "teuk_adjoint_step_n_async", "teuk_spin_tangent_workspace_bytes",
            "teuk_enable_spin_tangent", "teuk_set_spin_tangent", "teuk_get_spin_tangent", "teuk_step_n_spin_tangent",
            "teuk_spin_gradient")


def _check(rc):
    if rc != TEUK_OK:
        raise TeukError(rc, teuk_last_error())
    return rc


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def teuk_last_error():
    return _lib.teuk_last_error().decode()


def make_params(a, s, m, nr, ntheta, rstar_min, rstar_max, dt, coef_mode=TEUK_COEF_KERR,
                extract_rstar=(), extract_theta=(), stable_steps=0):
    er = np.ascontiguousarray(extract_rstar, dtype=np.float64).ravel()
    et = np.ascontiguousarray(extract_theta, dtype=np.float64).ravel()
    if er.shape != et.shape:
        raise ValueError("extraction coordinate arrays differ in length")
    p = teuk_params(float(a), int(s), int(m), int(nr), int(ntheta), float(rstar_min), float(rstar_max),
                    float(dt), int(coef_mode), int(er.size), None, None, int(stable_steps))
    if er.size:
        p.extract_rstar = er.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        p.extract_theta = et.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p._keep = (er, et)  # keep the host arrays alive as long as the struct
    return p


def teuk_workspace_bytes(p):
    n = _lib.teuk_workspace_bytes(ctypes.byref(p))
    if n == 0:
        raise TeukError(TEUK_E_INVALID_ARG, teuk_last_error())
    return n


def teuk_suggest_dt(p, n_steps, growth=10.0, courant=0.5):
    out = ctypes.c_double()
    _check(_lib.teuk_suggest_dt(ctypes.byref(p), int(n_steps), float(growth), float(courant), ctypes.byref(out)))
    return out.value


def teuk_init_grid(p, stream_handle, workspace):
    h = ctypes.c_void_p()
    _check(_lib.teuk_init_grid(ctypes.byref(p), ctypes.c_void_p(stream_handle), _dptr(workspace),
                               workspace.numel() * workspace.element_size(), ctypes.byref(h)))
    return h


def teuk_set_coefficients(h, ci, ch):
    return _check(_lib.teuk_set_coefficients(h, _dptr(ci), _dptr(ch)))


def teuk_set_initial_data(h, phi, pi):
    return _check(_lib.teuk_set_initial_data(h, _dptr(phi), _dptr(pi)))


def teuk_step_n(h, n, series=None):
    return _check(_lib.teuk_step_n(h, int(n), _dptr(series)))


def teuk_extract(h, rstar, theta, out):
    r = np.ascontiguousarray(rstar, dtype=np.float64).ravel()
    t = np.ascontiguousarray(theta, dtype=np.float64).ravel()
    if r.shape != t.shape:
        raise ValueError("coordinate arrays differ in length")
    return _check(_lib.teuk_extract(h, int(r.size), r.ctypes.data_as(ctypes.c_void_p),
                                    t.ctypes.data_as(ctypes.c_void_p), _dptr(out)))


def teuk_extract_noalloc(h, rstar, theta, out):
    r = np.ascontiguousarray(rstar, dtype=np.float64).ravel()
    t = np.ascontiguousarray(theta, dtype=np.float64).ravel()
    if r.shape != t.shape:
        raise ValueError("coordinate arrays differ in length")
    return _check(_lib.teuk_extract_noalloc(h, int(r.size), r.ctypes.data_as(ctypes.c_void_p),
                                            t.ctypes.data_as(ctypes.c_void_p), _dptr(out)))


def teuk_get_state(h, phi, pi):
    return _check(_lib.teuk_get_state(h, _dptr(phi), _dptr(pi)))


def teuk_check_finite(h):
    rc = _lib.teuk_check_finite(h)
    if rc == TEUK_E_NONFINITE:
        return False
    _check(rc)
    return True


def teuk_steps_taken(h):
    return _lib.teuk_steps_taken(h)


def teuk_get_dt(h):
    return _lib.teuk_get_dt(h)


def teuk_set_tile(h, rows_per_tile, waves_per_block):
    return _check(_lib.teuk_set_tile(h, int(rows_per_tile), int(waves_per_block)))


def teuk_get_tile(h):
    r, w = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.teuk_get_tile(h, ctypes.byref(r), ctypes.byref(w)))
    return r.value, w.value


def teuk_set_steps_per_pass(h, steps_per_pass):
    return _check(_lib.teuk_set_steps_per_pass(h, int(steps_per_pass)))


TEUK_CACHE_AUTO, TEUK_CACHE_KEEP, TEUK_CACHE_STREAM = 0, 1, 2


def teuk_set_cache_policy(h, policy):
    return _check(_lib.teuk_set_cache_policy(h, int(policy)))


def teuk_get_cache_policy(h):
    """(policy, keeps): the policy and whether states are currently kept in cache."""
    p, k = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.teuk_get_cache_policy(h, ctypes.byref(p), ctypes.byref(k)))
    return p.value, bool(k.value)


def teuk_get_steps_per_pass(h):
    v = ctypes.c_int32()
    _check(_lib.teuk_get_steps_per_pass(h, ctypes.byref(v)))
    return v.value


def teuk_set_block_launch(h, steps, cols=0):
    return _check(_lib.teuk_set_block_launch(h, int(steps), int(cols)))


def teuk_get_block_launch(h):
    """(steps, cols) of the block pass (cols 0: unset)."""
    k, c = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.teuk_get_block_launch(h, ctypes.byref(k), ctypes.byref(c)))
    return k.value, c.value


def teuk_set_finite_check(h, every):
    return _check(_lib.teuk_set_finite_check(h, int(every)))


def teuk_set_adjoint_tile(h, rows_per_tile, waves_per_block):
    return _check(_lib.teuk_set_adjoint_tile(h, int(rows_per_tile), int(waves_per_block)))


def teuk_get_adjoint_tile(h):
    r, w = ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.teuk_get_adjoint_tile(h, ctypes.byref(r), ctypes.byref(w)))
    return r.value, w.value


def teuk_free(h):
    return _check(_lib.teuk_free(h))


def teuk_window_bytes(h, n):
    nb = _lib.teuk_window_bytes(h, int(n))
    if nb == 0 and n > 0:
        raise TeukError(TEUK_E_INVALID_ARG, teuk_last_error())
    return nb


def teuk_step_n_store(h, n, series, window):
    return _check(_lib.teuk_step_n_store(h, int(n), _dptr(series), _dptr(window)))


def teuk_step_n_tangent(h, n, window):
    return _check(_lib.teuk_step_n_tangent(h, int(n), _dptr(window)))


def teuk_spin_tangent_workspace_bytes(h):
    return int(_lib.teuk_spin_tangent_workspace_bytes(h))


def teuk_enable_spin_tangent(h, workspace):
    return _check(_lib.teuk_enable_spin_tangent(h, _dptr(workspace), workspace.numel() * workspace.element_size()))


def teuk_set_spin_tangent(h, vphi, vpi):
    return _check(_lib.teuk_set_spin_tangent(h, _dptr(vphi), _dptr(vpi)))


def teuk_get_spin_tangent(h, vphi, vpi):
    return _check(_lib.teuk_get_spin_tangent(h, _dptr(vphi), _dptr(vpi)))


def teuk_step_n_spin_tangent(h, n, series, tseries):
    return _check(_lib.teuk_step_n_spin_tangent(h, int(n), _dptr(series), _dptr(tseries)))


def teuk_spin_gradient(h, n, dseries, tseries, accum):
    """accum (one-element float64 device tensor) += sum Re(conj(dseries) tseries); asynchronous."""
    return _check(_lib.teuk_spin_gradient(h, int(n), _dptr(dseries), _dptr(tseries), _dptr(accum)))


def teuk_get_window_slot(h, window, k, phi, pi):
    return _check(_lib.teuk_get_window_slot(h, _dptr(window), int(k), _dptr(phi), _dptr(pi)))


def teuk_source_workspace_bytes(h):
    nb = _lib.teuk_source_workspace_bytes(h)
    if nb == 0:
        raise TeukError(TEUK_E_INVALID_ARG, teuk_last_error())
    return nb


def teuk_set_source(h, workspace, gi, gh):
    nb = workspace.numel() * workspace.element_size() if workspace is not None else 0
    return _check(_lib.teuk_set_source(h, _dptr(workspace), nb, _dptr(gi), _dptr(gh)))


def teuk_step_n_source(h, n, series, f):
    """f: host array of n x 2 complex time factors (f(t_k), f(t_k + dt/2))."""
    fa = np.ascontiguousarray(np.asarray(f, dtype=np.complex128).reshape(int(n), 2)).view(np.float64)
    return _check(_lib.teuk_step_n_source(h, int(n), _dptr(series), fa.ctypes.data_as(ctypes.c_void_p)))


def teuk_adjoint_workspace_bytes(h):
    nb = _lib.teuk_adjoint_workspace_bytes(h)
    if nb == 0:
        raise TeukError(TEUK_E_INVALID_ARG, teuk_last_error())
    return nb


def teuk_enable_adjoint(h, workspace):
    return _check(_lib.teuk_enable_adjoint(h, _dptr(workspace), workspace.numel() * workspace.element_size()))


def teuk_adjoint_step_n(h, n, lam_phi, lam_pi, dseries, window, flags=0, spin=True):
    """Returns this segment's contribution to dL/da (None with spin=False, when
    only the cotangents are computed and window may be None); lam_phi, lam_pi
    are updated in place."""
    acc = ctypes.c_double(0.0)
    _check(_lib.teuk_adjoint_step_n(h, int(n), _dptr(lam_phi), _dptr(lam_pi), _dptr(dseries), _dptr(window),
                                    int(flags), ctypes.byref(acc) if spin else None))
    return acc.value if spin else None


def teuk_adjoint_step_n_async(h, n, lam_phi, lam_pi, dseries, window, flags, accum):
    """As teuk_adjoint_step_n with dL/da added to the device float64 tensor
    `accum` (one element) on the grid's stream; no synchronisation."""
    return _check(_lib.teuk_adjoint_step_n_async(h, int(n), _dptr(lam_phi), _dptr(lam_pi), _dptr(dseries),
                                                 _dptr(window), int(flags), _dptr(accum)))


def _aligned_bytes(torch, nbytes, device):
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + nbytes]


def _cuda_device(torch, device):
    """The device with its index filled in (the current one for "cuda" or None)."""
    d = torch.device(device) if device is not None else torch.device("cuda")
    if d.index is None:
        d = torch.device(d.type, torch.cuda.current_device())
    return d


class TeukGrid:
    """One grid on the current CUDA/HIP device: owns its workspace tensor.

    Field tensors are torch.complex128 of shape (ntheta, nr) on the device."""

    def __init__(self, a, s, m, nr, ntheta, rstar_min, rstar_max, dt, coef_mode=TEUK_COEF_KERR,
                 extract_rstar=(), extract_theta=(), device=None, stream=None, stable_steps=0):
        import torch

        self.torch = torch
        self.device = _cuda_device(torch, device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.params = make_params(a, s, m, nr, ntheta, rstar_min, rstar_max, dt, coef_mode,
                                  extract_rstar, extract_theta, stable_steps)
        self.nr, self.ntheta = int(nr), int(ntheta)
        self.n_extract = self.params.n_extract
        nbytes = teuk_workspace_bytes(self.params)
        self.workspace = _aligned_bytes(torch, nbytes, self.device)
        self.adjoint_workspace = None
        self.spin_tangent_workspace = None
        with torch.cuda.device(self.device):
            self.handle = teuk_init_grid(self.params, self.stream.cuda_stream, self.workspace)

    @property
    def shape(self):
        return (self.ntheta, self.nr)

    @property
    def dt(self):
        return teuk_get_dt(self.handle)

    @property
    def steps(self):
        return teuk_steps_taken(self.handle)

    def _field(self, t):
        t = self.torch.as_tensor(t, dtype=self.torch.complex128, device=self.device)
        if tuple(t.shape) != self.shape:
            raise ValueError(f"expected shape {self.shape}, got {tuple(t.shape)}")
        return t.contiguous()

    def set_coefficients(self, ci, ch):
        ci = self.torch.as_tensor(ci, dtype=self.torch.float64, device=self.device).contiguous()
        ch = self.torch.as_tensor(ch, dtype=self.torch.float64, device=self.device).contiguous()
        if ci.numel() != TEUK_NCOEF * self.ntheta * self.nr or ch.numel() != TEUK_NCOEF * self.ntheta * (self.nr - 1):
            raise ValueError("coefficient tables have the wrong size")
        self._coef_keep = (ci, ch)
        teuk_set_coefficients(self.handle, ci, ch)

    def set_initial_data(self, phi, pi):
        phi, pi = self._field(phi), self._field(pi)
        self._init_keep = (phi, pi)
        teuk_set_initial_data(self.handle, phi, pi)

    def step(self, n, series=True):
        """n steps; returns the extraction series (n, n_extract) complex128 or None."""
        out = None
        if series and self.n_extract > 0 and n > 0:
            out = self.torch.empty((int(n), self.n_extract), dtype=self.torch.complex128, device=self.device)
        teuk_step_n(self.handle, n, out)
        return out

    def state(self):
        phi = self.torch.empty(self.shape, dtype=self.torch.complex128, device=self.device)
        pi = self.torch.empty_like(phi)
        teuk_get_state(self.handle, phi, pi)
        return phi, pi

    def extract(self, rstar, theta):
        n = int(np.asarray(rstar).size)
        out = self.torch.empty(n, dtype=self.torch.complex128, device=self.device)
        teuk_extract(self.handle, rstar, theta, out)
        return out

    # ---- adjoint ---------------------------------------------------------
    def enable_adjoint(self):
        if self.adjoint_workspace is None:
            ws = _aligned_bytes(self.torch, teuk_adjoint_workspace_bytes(self.handle), self.device)
            teuk_enable_adjoint(self.handle, ws)
            self.adjoint_workspace = ws

    def enable_spin_tangent(self):
        """Carry v = du/da beside the state (forward-mode spin derivative); v = 0."""
        self.enable_adjoint()
        if self.spin_tangent_workspace is None:
            ws = _aligned_bytes(self.torch, teuk_spin_tangent_workspace_bytes(self.handle), self.device)
            teuk_enable_spin_tangent(self.handle, ws)
            self.spin_tangent_workspace = ws

    def set_spin_tangent(self, vphi=None, vpi=None):
        """v from (ntheta, nr) complex128 tensors, or v = 0."""
        self.enable_spin_tangent()
        if vphi is None and vpi is None:
            teuk_set_spin_tangent(self.handle, None, None)
            return
        vphi = self.torch.as_tensor(vphi, dtype=self.torch.complex128, device=self.device).contiguous()
        vpi = self.torch.as_tensor(vpi, dtype=self.torch.complex128, device=self.device).contiguous()
        if tuple(vphi.shape) != self.shape or tuple(vpi.shape) != self.shape:
            raise ValueError(f"v must have shape {self.shape}")
        self._v_keep = (vphi, vpi)  # until the stream has read them
        teuk_set_spin_tangent(self.handle, vphi, vpi)

    def spin_tangent(self):
        """The current v as (phi, pi) tensors of shape (ntheta, nr)."""
        phi = self.torch.empty(self.shape, dtype=self.torch.complex128, device=self.device)
        pi = self.torch.empty_like(phi)
        teuk_get_spin_tangent(self.handle, phi, pi)
        return phi, pi

    def step_spin_tangent(self, n, series=True):
        """n steps of u and v; returns (series of u, series of v), each (n, n_extract)
        complex128 (None without extraction points or with series=False)."""
        s = t = None
        if series and self.n_extract > 0:
            s = self.torch.empty((int(n), self.n_extract), dtype=self.torch.complex128, device=self.device)
            t = self.torch.empty_like(s)
        teuk_step_n_spin_tangent(self.handle, n, s, t)
        return s, t

    def new_window(self, n):
        """Device buffer for n stored states."""
        return _aligned_bytes(self.torch, max(teuk_window_bytes(self.handle, n), 1), self.device)

    def step_store(self, n, window, series=True):
        out = None
        if series and self.n_extract > 0 and n > 0:
            out = self.torch.empty((int(n), self.n_extract), dtype=self.torch.complex128, device=self.device)
        teuk_step_n_store(self.handle, n, out, window)
        return out

    def step_tangent(self, n, window):
        """n steps, leaving T_k = (dA/da) u^k in window slot k (teuk_step_n_tangent)."""
        self.enable_adjoint()
        teuk_step_n_tangent(self.handle, n, window)

    def set_source(self, gi, gh):
        """Source profile g of the inhomogeneous variant, at integer (ntheta, nr)
        and half (ntheta, nr-1) positions (complex128); None, None detaches."""
        if gi is None and gh is None:
            teuk_set_source(self.handle, None, None, None)
            return
        gi = self.torch.as_tensor(gi, dtype=self.torch.complex128, device=self.device).contiguous()
        gh = self.torch.as_tensor(gh, dtype=self.torch.complex128, device=self.device).contiguous()
        if tuple(gi.shape) != self.shape or tuple(gh.shape) != (self.ntheta, self.nr - 1):
            raise ValueError("source profiles must have shapes (ntheta, nr) and (ntheta, nr - 1)")
        if getattr(self, "source_workspace", None) is None:
            self.source_workspace = _aligned_bytes(self.torch, teuk_source_workspace_bytes(self.handle), self.device)
        self._source_keep = (gi, gh)  # until the stream has passed the copy
        teuk_set_source(self.handle, self.source_workspace, gi, gh)

    def step_source(self, f, series=True):
        """len(f) steps with the source; f[k] = (f(t_k), f(t_k + dt/2)).  Returns the series or None."""
        f = np.asarray(f, dtype=np.complex128)
        n = int(f.shape[0])
        out = None
        if series and self.n_extract > 0 and n > 0:
            out = self.torch.empty((n, self.n_extract), dtype=self.torch.complex128, device=self.device)
        teuk_step_n_source(self.handle, n, out, f)
        return out

    def window_slot(self, window, k):
        """Slot k of a window as (phi, pi) tensors of shape (ntheta, nr)."""
        phi = self.torch.empty(self.shape, dtype=self.torch.complex128, device=self.device)
        pi = self.torch.empty_like(phi)
        teuk_get_window_slot(self.handle, window, k, phi, pi)
        return phi, pi

    def adjoint(self, n, lam_phi, lam_pi, dseries, window, project_initial=False, spin=True, tangent=False,
                accum=None):
        """Reverse of n stored steps; updates (lam_phi, lam_pi) in place, returns the dL/da part
        (spin=False: cotangents only, window may be None, returns None).  tangent: the window
        holds step tangents (step_tangent) instead of states (step_store).  accum: a one-element
        float64 device tensor to which dL/da is added without synchronising (returns None)."""
        self.enable_adjoint()
        if dseries is not None:
            dseries = self.torch.as_tensor(dseries, dtype=self.torch.complex128, device=self.device).contiguous()
            if tuple(dseries.shape) != (int(n), self.n_extract):
                raise ValueError("dseries must have shape (n, n_extract)")
        flags = (TEUK_ADJ_PROJECT_INITIAL if project_initial else 0) | (TEUK_ADJ_TANGENT_WINDOW if tangent else 0)
        if accum is not None:
            if accum.dtype != self.torch.float64 or accum.numel() != 1 or accum.device != self.device:
                raise ValueError("accum must be a one-element float64 tensor on the grid's device")
            teuk_adjoint_step_n_async(self.handle, n, lam_phi, lam_pi, dseries, window, flags, accum)
            return None
        return teuk_adjoint_step_n(self.handle, n, lam_phi, lam_pi, dseries, window, flags, spin)

    def check_finite(self):
        return teuk_check_finite(self.handle)

    def set_tile(self, rows_per_tile, waves_per_block):
        teuk_set_tile(self.handle, rows_per_tile, waves_per_block)

    def tile(self):
        return teuk_get_tile(self.handle)

    def set_steps_per_pass(self, steps_per_pass):
        teuk_set_steps_per_pass(self.handle, steps_per_pass)

    def steps_per_pass(self):
        return teuk_get_steps_per_pass(self.handle)

    def set_block_launch(self, steps, cols=0):
        """Small-grid block pass: steps per launch (0: off) and columns a
        workgroup holds (0: keep the grid's)."""
        teuk_set_block_launch(self.handle, steps, cols)

    def block_launch(self):
        return teuk_get_block_launch(self.handle)

    def set_block_steps(self, steps):
        """Steps per launch of the block pass with the grid's columns (0: off)."""
        teuk_set_block_launch(self.handle, steps, 0)

    def block_steps(self):
        return teuk_get_block_launch(self.handle)[0]

    def set_cache_policy(self, policy):
        teuk_set_cache_policy(self.handle, policy)

    def cache_policy(self):
        return teuk_get_cache_policy(self.handle)

    def set_finite_check(self, every):
        """Device check of the state every `every` steps inside step(); 0: off."""
        teuk_set_finite_check(self.handle, every)

    def set_adjoint_tile(self, rows_per_tile, waves_per_block):
        teuk_set_adjoint_tile(self.handle, rows_per_tile, waves_per_block)

    def adjoint_tile(self):
        return teuk_get_adjoint_tile(self.handle)

    def close(self):
        if getattr(self, "handle", None) is not None:
            teuk_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class TeukBatch:
    """Many grids advanced by one persistent launch per step (C ABI teuk_batch_*).

    members: list of dicts with a, s, m, nr, ntheta, rstar_min, rstar_max, dt and
    optionally extract_rstar, extract_theta."""

    def __init__(self, members, device=None, stream=None):
        import torch

        self.torch = torch
        self.device = _cuda_device(torch, device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.members = [dict(m) for m in members]
        arr = (teuk_params * len(members))()
        keep = []
        for k, m in enumerate(members):
            p = make_params(m["a"], m["s"], m["m"], m["nr"], m["ntheta"], m["rstar_min"], m["rstar_max"], m["dt"],
                            extract_rstar=m.get("extract_rstar", ()), extract_theta=m.get("extract_theta", ()),
                            stable_steps=m.get("stable_steps", 0))
            keep.append(p._keep)  # the extraction coordinate arrays the copied structs point to
            arr[k] = p
        self._arr, self._keep = arr, keep
        nb = _lib.teuk_batch_workspace_bytes(arr, len(members))
        if nb == 0:
            raise TeukError(TEUK_E_INVALID_ARG, teuk_last_error())
        self.workspace = _aligned_bytes(torch, nb, self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib.teuk_batch_init(arr, len(members), ctypes.c_void_p(self.stream.cuda_stream),
                                        _dptr(self.workspace), nb, ctypes.byref(h)))
        self.handle = h

    def __len__(self):
        return len(self.members)

    def shape(self, k):
        return (int(self.members[k]["ntheta"]), int(self.members[k]["nr"]))

    def set_initial_data(self, k, phi, pi):
        phi = self.torch.as_tensor(phi, dtype=self.torch.complex128, device=self.device).contiguous()
        pi = self.torch.as_tensor(pi, dtype=self.torch.complex128, device=self.device).contiguous()
        if tuple(phi.shape) != self.shape(k) or tuple(pi.shape) != self.shape(k):
            raise ValueError(f"member {k}: expected shape {self.shape(k)}")
        self._keep = getattr(self, "_keep", {})
        self._keep[k] = (phi, pi)
        _check(_lib.teuk_batch_set_initial_data(self.handle, int(k), _dptr(phi), _dptr(pi)))

    def state(self, k):
        phi = self.torch.empty(self.shape(k), dtype=self.torch.complex128, device=self.device)
        pi = self.torch.empty_like(phi)
        _check(_lib.teuk_batch_get_state(self.handle, int(k), _dptr(phi), _dptr(pi)))
        return phi, pi

    def step(self, n):
        _check(_lib.teuk_batch_step_n(self.handle, int(n)))

    def set_launch(self, rows_per_tile, waves_per_block, n_blocks):
        _check(_lib.teuk_batch_set_launch(self.handle, int(rows_per_tile), int(waves_per_block), int(n_blocks)))

    def set_steps_per_pass(self, steps_per_pass):
        _check(_lib.teuk_batch_set_steps_per_pass(self.handle, int(steps_per_pass)))

    def n_extract(self):
        return int(_lib.teuk_batch_n_extract(self.handle))

    def extract(self, out=None):
        """Samples of all members' extraction points (complex128, member order)."""
        if out is None:
            out = self.torch.empty(self.n_extract(), dtype=self.torch.complex128, device=self.device)
        _check(_lib.teuk_batch_extract(self.handle, _dptr(out)))
        return out

    def launch(self):
        r, w, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.teuk_batch_get_launch(self.handle, ctypes.byref(r), ctypes.byref(w), ctypes.byref(b)))
        return r.value, w.value, b.value

    def total_points(self):
        return int(_lib.teuk_batch_total_points(self.handle))

    def close(self):
        if getattr(self, "handle", None) is not None:
            _check(_lib.teuk_batch_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def teuk_radius(a, rstar):
    """Boyer-Lindquist radius at tortoise coordinate rstar (M = 1)."""
    r = ctypes.c_double()
    _check(_lib.teuk_radius(float(a), float(rstar), ctypes.byref(r)))
    return r.value


def teuk_assemble_modes(samples, m_values, phi, r, psi, stream):
    """psi[k][o] = r_o^3 sum_j e^{i m_j phi_o} samples[k][j][o] (device tensors)."""
    m = np.ascontiguousarray(m_values, dtype=np.int32)
    ph = np.ascontiguousarray(phi, dtype=np.float64)
    rr = np.ascontiguousarray(r, dtype=np.float64)
    n_samples = int(samples.shape[0]) if samples.dim() == 3 else 0
    _check(_lib.teuk_assemble_modes(n_samples, int(m.size), m.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                    int(ph.size), ph.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    rr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _dptr(samples), _dptr(psi),
                                    ctypes.c_void_p(stream.cuda_stream)))
    return psi


def suggest_dt(a, s, m, nr, ntheta, rstar_min, rstar_max, n_steps, growth=10.0, courant=0.5):
    p = make_params(a, s, m, nr, ntheta, rstar_min, rstar_max, 1.0)
    return teuk_suggest_dt(p, n_steps, growth, courant)


__all__ = [n for n in EXPORTED] + ["TeukGrid", "TeukBatch", "TeukError", "make_params", "suggest_dt", "teuk_params"]

