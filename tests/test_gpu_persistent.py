"""The persistent launch of the step loop (teuk_set_persistent): runs of
two-step passes in one cooperative launch with a grid barrier between
passes.  The per-point arithmetic is that of the two-step kernel, so every
state and series must equal, bit for bit, the run with one launch per pass
(mode 0), and hence the oracle within the forward tolerance."""
import math

import numpy as np
import pytest
import torch

from paper_1010_3816_amd import inputs
from parity import rel_err, run_oracle, small_case

pytestmark = pytest.mark.gpu
TOL = 1e-11


def _run(gpu, w, phi0, pi0, calls, mode, tile=None, coef=None):
    """State and concatenated series after stepping `calls` = (n1, n2, ...)."""
    g = gpu.TeukGrid(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["dt"],
                     coef_mode=gpu.TEUK_COEF_USER if coef is not None else gpu.TEUK_COEF_KERR,
                     extract_rstar=w.get("extract_rstar", []), extract_theta=w.get("extract_theta", []))
    if coef is not None:
        g.set_coefficients(torch.from_numpy(coef[0]).cuda(), torch.from_numpy(coef[1]).cuda())
    if tile is not None:
        g.set_tile(*tile)
    g.set_persistent(mode)
    g.set_initial_data(torch.from_numpy(phi0).cuda(), torch.from_numpy(pi0).cuda())
    series = []
    for n in calls:
        s = g.step(n)
        if s is not None:
            series.append(s.cpu().numpy())
    assert g.check_finite()
    out = [t.cpu().numpy() for t in g.state()]
    g.close()
    return out[0], out[1], (np.concatenate(series) if series else None)


CASES = [
    # a, s, m, nr, nth, extraction points, tile, calls
    (0.0, -2, 2, 400, 32, ((100.0, math.pi / 2),), None, (1000,)),
    (0.7, -2, 1, 130, 20, ((20.0, 1.1),), (1, 1), (9, 4, 1, 6)),
    (0.9, 0, -3, 187, 70, (), (8, 4), (17,)),
    (0.99, -1, 4, 64, 9, ((5.0, 0.2), (15.0, 2.9)), (3, 2), (5, 5, 2)),
    (0.3, 0, 0, 3, 2, ((0.5, 1.0),), (1, 1), (8,)),
    (0.5, -2, 2, 500, 33, ((20.0, math.pi / 2),), (33, 4), (12,)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_persistent_bit_identical(gpu, case):
    a, s, m, nr, nth, ext, tile, calls = CASES[case]
    w = small_case(a, s, m, nr, nth, ext=ext)
    if case == 0:
        w = inputs.workload("schwarzschild_400x32")
    phi0, pi0 = inputs.random_state(nr, nth, seed=100 + case)
    ref = _run(gpu, w, phi0, pi0, calls, 0, tile)
    got = _run(gpu, w, phi0, pi0, calls, 1, tile)
    for k in range(3):
        if ref[k] is None:
            assert got[k] is None
        else:
            assert np.array_equal(got[k], ref[k]), (case, k)
    if nr * nth <= 20000:
        o = run_oracle(w, phi0, pi0, sum(calls))
        assert rel_err(ref[0], o[0]) <= TOL and rel_err(ref[1], o[1]) <= TOL
        if ref[2] is not None:
            assert rel_err(ref[2], o[2]) <= TOL


def test_persistent_user_coefficients(gpu):
    nr, nth = 90, 13
    rng = np.random.default_rng(12)
    ci = rng.uniform(-0.5, 0.5, (9, nth, nr))
    ch = rng.uniform(-0.5, 0.5, (9, nth, nr - 1))
    ci[0] += 1.0
    ch[0] += 1.0
    w = dict(a=0.0, s=0, m=1, nr=nr, ntheta=nth, rstar_min=0.0, rstar_max=30.0, dt=0.01,
             extract_rstar=[12.3], extract_theta=[0.7])
    phi0, pi0 = inputs.random_state(nr, nth, seed=5)
    ref = _run(gpu, w, phi0, pi0, (12,), 0, coef=(ci, ch))
    got = _run(gpu, w, phi0, pi0, (12,), 1, coef=(ci, ch))
    for k in range(3):
        assert np.array_equal(got[k], ref[k]), k


def test_persistent_modes_and_fallback(gpu):
    """Mode validation; a grid whose tiles do not fit one round runs with
    one launch per pass under mode 1 and gives the same result."""
    w = small_case(0.5, -2, 2, 400, 32)
    g = gpu.TeukGrid(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["dt"])
    assert g.persistent() == 0
    for bad in (-1, 2):
        with pytest.raises(RuntimeError):
            g.set_persistent(bad)
    g.close()
    # 1-row tiles of a 6400 x 256 grid: 27,392 wavefronts, more than one round
    w = small_case(0.5, -2, 2, 6400, 256, rmin=-100.0, rmax=600.0)
    phi0, pi0 = inputs.random_state(6400, 256, seed=7)
    ref = _run(gpu, w, phi0, pi0, (6,), 0, (1, 4))
    got = _run(gpu, w, phi0, pi0, (6,), 1, (1, 4))
    for k in range(3):
        assert np.array_equal(got[k], ref[k]), k
