"""CPU tests of the C-ABI boundary: the library loads, exports every symbol
declared in include/teuk.h, and rejects invalid arguments on the host before
touching a device."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "teuk.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(teuk_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def b():
    import __graft_entry__ as ge
    from paper_1010_3816_amd import build

    if not os.path.exists(build.LIB):
        ge.build_hip()
    from paper_1010_3816_amd import binding

    return binding


def test_every_declared_symbol_is_exported(b):
    lib = ctypes.CDLL(b.LIB_PATH)
    names = _declared_symbols()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) <= set(b.EXPORTED)


def test_workspace_bytes_and_validation(b):
    p = b.make_params(0.9, -2, 2, 6400, 256, -100.0, 600.0, 1e-3, extract_rstar=[500.0], extract_theta=[math.pi / 2])
    n = b.teuk_workspace_bytes(p)
    assert n >= 4 * 6400 * 256 * 16
    bad = [
        dict(a=1.0), dict(a=-0.1), dict(s=3), dict(nr=2), dict(ntheta=1), dict(rstar_min=5.0, rstar_max=5.0),
        dict(dt=float("nan")), dict(dt=float("inf")), dict(dt=0.0, coef_mode=b.TEUK_COEF_USER),
    ]
    base = dict(a=0.5, s=-2, m=2, nr=100, ntheta=8, rstar_min=-10.0, rstar_max=10.0, dt=0.01)
    for kw in bad:
        args = dict(base, **kw)
        with pytest.raises(b.TeukError) as ei:
            b.teuk_workspace_bytes(b.make_params(**args))
        assert ei.value.code == b.TEUK_E_INVALID_ARG
    with pytest.raises(b.TeukError):
        b.teuk_workspace_bytes(b.make_params(**base, extract_rstar=[11.0], extract_theta=[1.0]))
    with pytest.raises(b.TeukError):
        b.teuk_workspace_bytes(b.make_params(**base, extract_rstar=[0.0], extract_theta=[4.0]))


def test_init_rejects_before_device_work(b):
    lib = ctypes.CDLL(b.LIB_PATH)
    lib.teuk_init_grid.argtypes = [ctypes.POINTER(b.teuk_params), ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p)]
    p = b.make_params(0.5, -2, 2, 100, 8, -10.0, 10.0, 0.01)
    h = ctypes.c_void_p()
    # NULL workspace, misaligned workspace, too small workspace: all host-side errors
    assert lib.teuk_init_grid(ctypes.byref(p), None, None, 0, ctypes.byref(h)) == b.TEUK_E_INVALID_ARG
    assert lib.teuk_init_grid(ctypes.byref(p), None, ctypes.c_void_p(0x1001), 1 << 30,
                              ctypes.byref(h)) == b.TEUK_E_WORKSPACE
    assert lib.teuk_init_grid(ctypes.byref(p), None, ctypes.c_void_p(0x100000), 16,
                              ctypes.byref(h)) == b.TEUK_E_WORKSPACE
    assert "workspace" in b.teuk_last_error()


def test_time_step_policy_and_strict_mode(b):
    """dt <= 0 takes the policy step (validation accepts it); with a horizon
    a given dt above the stability bound is rejected as TEUK_E_UNSTABLE_DT
    before any other argument is used (here: a NULL workspace)."""
    from paper_1010_3816_amd import inputs

    lib = ctypes.CDLL(b.LIB_PATH)
    lib.teuk_init_grid.argtypes = [ctypes.POINTER(b.teuk_params), ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p)]
    w = inputs.workload("schwarzschild_400x32")
    geo = (w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"])
    h = ctypes.c_void_p()
    assert b.teuk_workspace_bytes(b.make_params(*geo, 0.0)) > 0
    bound = b.suggest_dt(*geo, 1000, 10.0, 1.0)
    # the literal dt = 0.5 dr* of this workload is far above the bound (S14)
    assert 0.5 * w["dr"] > 5 * bound
    cases = [(0.5 * w["dr"], 1000, b.TEUK_E_UNSTABLE_DT), (bound * 1.001, 1000, b.TEUK_E_UNSTABLE_DT),
             (bound * 0.999, 1000, b.TEUK_E_INVALID_ARG), (0.5 * w["dr"], 0, b.TEUK_E_INVALID_ARG),
             (0.0, 1000, b.TEUK_E_INVALID_ARG), (-1.0, 0, b.TEUK_E_INVALID_ARG)]
    for dt, horizon, rc in cases:
        p = b.make_params(*geo, dt, stable_steps=horizon)
        # INVALID_ARG: the step passed, then the NULL workspace was refused
        assert lib.teuk_init_grid(ctypes.byref(p), None, None, 0, ctypes.byref(h)) == rc, (dt, horizon)
    assert "workspace" in b.teuk_last_error()
    p = b.make_params(*geo, 0.5 * w["dr"], stable_steps=1000)
    lib.teuk_init_grid(ctypes.byref(p), None, None, 0, ctypes.byref(h))
    assert "grow" in b.teuk_last_error()


def test_null_handle_errors(b):
    lib = ctypes.CDLL(b.LIB_PATH)
    lib.teuk_step_n.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    assert lib.teuk_step_n(None, 1, None) == b.TEUK_E_INVALID_ARG
    assert lib.teuk_free(None) == b.TEUK_OK


def test_suggest_dt_host_only(b):
    from paper_1010_3816_amd import inputs

    w = inputs.workload("schwarzschild_400x32")
    dt = b.suggest_dt(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["steps"])
    assert 0.0 < dt < 0.5 * w["dr"]
    # longer runs need smaller steps; growth 10 over n steps scales as n^(-1/4)
    dt2 = b.suggest_dt(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"],
                       16 * w["steps"])
    assert dt2 == pytest.approx(dt / 2, rel=1e-12)


def test_radius_and_mode_sum_validation():
    """teuk_radius inverts the oracle's tortoise coordinate; the mode sum
    rejects bad sizes and observers before any device work."""
    import ctypes

    import oracle
    from paper_1010_3816_amd import binding as b

    for a, rs in [(0.0, 10.0), (0.9, -50.0), (0.99, 500.0), (0.5, 3.0), (0.7, -100.0)]:
        r = b.teuk_radius(a, rs)
        r_oracle = 1.0 + math.sqrt(1.0 - a * a) + oracle.tortoise_x(a, rs)
        assert abs(r - r_oracle) <= 4 * math.ulp(r_oracle), (a, rs, r, r_oracle)
    with pytest.raises(b.TeukError):
        b.teuk_radius(1.0, 5.0)
    with pytest.raises(b.TeukError):
        b.teuk_radius(0.5, float("nan"))
    m = (ctypes.c_int32 * 2)(1, 2)
    phi = (ctypes.c_double * 2)(0.0, 1.0)
    r_ok = (ctypes.c_double * 2)(10.0, 20.0)
    r_bad = (ctypes.c_double * 2)(10.0, 0.0)
    lib = b._lib
    assert lib.teuk_assemble_modes(1, 0, m, 2, phi, r_ok, None, None, None) == b.TEUK_E_INVALID_ARG
    assert lib.teuk_assemble_modes(1, 2, m, 65, phi, r_ok, None, None, None) == b.TEUK_E_INVALID_ARG
    assert lib.teuk_assemble_modes(1, 2, m, 2, phi, r_bad, None, None, None) == b.TEUK_E_INVALID_ARG
    assert lib.teuk_assemble_modes(1, 2, m, 2, phi, r_ok, None, None, None) == b.TEUK_E_INVALID_ARG  # NULL tensors
    assert lib.teuk_assemble_modes(0, 2, m, 2, phi, r_ok, None, None, None) == b.TEUK_OK  # nothing to do


def test_round_rows_fill_whole_rounds():
    """Autotuner candidates: tile heights whose tiles just fit k rounds of
    two wavefronts per SIMD (256 CUs: 2048 resident wavefronts)."""
    from paper_1010_3816_amd.autotune import round_rows

    # 25600 columns = 427 strips of 60; 512 rows cut into 4, 9, 14, 19 tiles
    assert round_rows(25600, 512, 256) == [27, 37, 57, 128]
    # 6400 columns = 107 strips: one round takes 19 tiles of 14 rows, two
    # rounds 38 of 7, three 57 of 5, four 76 of 4
    assert round_rows(6400, 256, 256) == [4, 5, 7, 14]
    assert round_rows(6400, 256, 256, lo=8) == [14]
    # k rounds hold the tiles, k - 1 rounds would not
    for nr, nth in ((25600, 512), (6400, 256), (12800, 128), (3000, 64)):
        strips = -(-nr // 60)
        for k in (1, 2, 3, 4):
            (r,) = round_rows(nr, nth, 256, rounds=(k,), lo=1, hi=nth)
            tiles = strips * -(-nth // r)
            assert tiles <= k * 2048, (nr, nth, k, r)
            assert r == 1 or strips * -(-nth // (r - 1)) > k * 2048, (nr, nth, k, r)


def test_block_candidates():
    """Autotuner candidates of the small-grid block pass: (steps, columns)
    for workgroups of up to 256, 512 and 1024 threads (at most 64 columns),
    at least 4 steps, and no more workgroups than CUs."""
    from paper_1010_3816_amd.autotune import block_candidates

    c400 = block_candidates(400, 32, 256)
    # 8 columns allow 3 steps at most: no candidate; 16 columns: 4..7 steps
    # (7 writes 2 columns a workgroup: 200 workgroups); 32 columns: 4..15
    assert [k for k, c in c400 if c == 16] == [4, 5, 6, 7]
    assert [k for k, c in c400 if c == 32] == list(range(4, 16))
    assert {c for _, c in c400} == {16, 32}
    # 3200 x 32 on 256 CUs: at least 13 written columns a workgroup
    assert max(k for k, c in block_candidates(3200, 32, 256) if c == 32) == 9
    assert not [k for k, c in block_candidates(3200, 32, 256) if c == 16]
    assert block_candidates(400, 65, 256) == [] and block_candidates(6400, 64, 256) == []
    for nr, nth in ((400, 32), (800, 32), (1600, 64), (130, 20), (3, 2)):
        for k, c in block_candidates(nr, nth, 256):
            assert 4 <= k <= (c - 2) // 2 and c * nth <= 1024 and c <= 64
            assert -(-nr // (c - 2 * k)) <= 256


def test_source_inputs():
    """The source-term inputs: profile shapes, the blob's peak at the column
    and row nearest its centre, the half-position samples between the
    columns' values, and the time factors (f(t_k), f(t_k + dt/2))."""
    import numpy as np

    from paper_1010_3816_amd import inputs

    nr, nth = 201, 32
    gi, gh = inputs.localised_source(nr, nth, -50.0, 150.0, 30.0, width=2.0)
    assert gi.shape == (nth, nr) and gh.shape == (nth, nr - 1)
    assert gi.dtype == np.complex128 and gh.dtype == np.complex128
    j, i = np.unravel_index(np.argmax(np.abs(gi)), gi.shape)
    assert i == 80 and j in (15, 16)  # r* = 30 is column 80; theta = pi/2 lies between rows 15 and 16
    # at the half positions the (concave near the peak) Gaussian exceeds the columns' mean there
    assert gh[j, 80] > 0.5 * (gi[j, 80] + gi[j, 81]).real and gh[j, 79] > 0.5 * (gi[j, 79] + gi[j, 80]).real
    # 41 or more units of r* from the centre: below exp(-41^2 / 8) ~ 6e-92
    assert np.max(np.abs(gi[:, :40])) < 1e-91 and np.max(np.abs(gh[:, 121:])) < 1e-91
    f = inputs.oscillating_factors(5, 0.1, omega=2.0, amplitude=3.0, t0=1.0)
    assert f.shape == (5, 2)
    assert np.allclose(f[2, 0], 3.0 * np.exp(2j * 1.2), rtol=0, atol=1e-15)
    assert np.allclose(f[2, 1], 3.0 * np.exp(2j * 1.25), rtol=0, atol=1e-15)
