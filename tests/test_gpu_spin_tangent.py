"""GPU forward-mode spin derivative (C ABI teuk_step_n_spin_tangent) against
the oracle's forward-mode evolution (oracle.OracleGrid.evolve_spin_tangent).

Bars: u, v and both sample series within the 1e-11 normwise relative
tolerance of the forward path; u and its series bit-identical to
teuk_step_n; dL/da within 1e-10 relative of the GPU reverse pass (two exact
routes whose rounding differs)."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1010_3816_amd import inputs
from parity import rel_err, small_case

pytestmark = pytest.mark.gpu
TOL = 1e-11


def _grid(gpu, w):
    return gpu.TeukGrid(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["dt"],
                        extract_rstar=w["extract_rstar"], extract_theta=w["extract_theta"])


def _run(gpu, w, u0, v0, n, tile=None):
    g = _grid(gpu, w)
    if tile is not None:
        g.set_adjoint_tile(*tile)
    g.set_initial_data(torch.from_numpy(u0[0]).cuda(), torch.from_numpy(u0[1]).cuda())
    if v0 is None:
        g.set_spin_tangent()
    else:
        g.set_spin_tangent(torch.from_numpy(v0[0]).cuda(), torch.from_numpy(v0[1]).cuda())
    s, t = g.step_spin_tangent(n)
    u = g.state()
    v = g.spin_tangent()
    torch.cuda.synchronize()
    out = [x.cpu().numpy() for x in (*u, *v)] + [None if s is None else s.cpu().numpy(),
                                                 None if t is None else t.cpu().numpy()]
    g.close()
    return out


def _oracle(w, u0, v0, n):
    o = oracle.OracleGrid(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["dt"])
    p, q = o.project(*u0)
    vp, vq = o.project(*v0) if v0 is not None else (np.zeros_like(p), np.zeros_like(q))
    return o.evolve_spin_tangent(p, q, vp, vq, n, w["extract_rstar"], w["extract_theta"])


@pytest.mark.parametrize("a,s,m,nr,nth,n,tile", [
    (0.7, -2, 2, 150, 24, 7, None),      # ragged last strip, odd step count
    (0.4, -2, 1, 130, 20, 6, (5, 2)),    # odd |m| (anti-mirror ghosts), short tiles
    (0.9, 0, -3, 187, 70, 5, (16, 4)),   # several chunks with a ragged last one
    (0.99, -1, 4, 64, 9, 4, (3, 1)),
    (0.5, 2, 0, 3, 2, 3, (1, 1)),        # smallest grid: one interior column, pole rows only
])
def test_parity_with_oracle(gpu, a, s, m, nr, nth, n, tile):
    w = small_case(a, s, m, nr, nth, ext=((20.0, math.pi / 2), (-12.0, 0.3)))
    u0 = inputs.random_state(nr, nth, seed=nr + 3 * nth)
    v0 = inputs.random_state(nr, nth, seed=nr + 3 * nth + 1)
    g = _run(gpu, w, u0, v0, n, tile)
    o = _oracle(w, u0, v0, n)
    for k in range(6):
        assert rel_err(g[k], o[k]) <= TOL, k
    assert np.max(np.abs(o[5])) > 0


@pytest.mark.parametrize("spp", [1, 2])
def test_state_bit_identical_to_step(gpu, spp):
    """u and its series are those of teuk_step_n, bit for bit."""
    w = small_case(0.6, -2, 2, 170, 26, ext=((20.0, math.pi / 2),))
    u0 = inputs.random_state(170, 26, seed=31)
    g = _grid(gpu, w)
    g.set_steps_per_pass(spp)
    g.set_initial_data(torch.from_numpy(u0[0]).cuda(), torch.from_numpy(u0[1]).cuda())
    ser = g.step(9).cpu().numpy()
    ref = [x.cpu().numpy() for x in g.state()]
    g.close()
    out = _run(gpu, w, u0, None, 9)
    assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1])
    assert np.array_equal(out[4], ser)


def test_extraction_fallback(gpu):
    """Two extraction points in one tile: the samples come from separate
    passes, with the same values as the fused ones."""
    ext = ((20.0, math.pi / 2), (20.5, math.pi / 2 + 0.1), (-3.0, 1.0))
    w = small_case(0.6, -2, 2, 150, 24, ext=ext)
    u0 = inputs.random_state(150, 24, seed=41)
    v0 = inputs.random_state(150, 24, seed=42)
    g = _run(gpu, w, u0, v0, 6)
    o = _oracle(w, u0, v0, 6)
    for k in range(6):
        assert rel_err(g[k], o[k]) <= TOL, k


def test_forward_and_reverse_spin_gradient_agree(gpu):
    """dL/da = sum Re(conj(dL/ds) ds/da) from the forward mode equals the
    reverse pass's (stored-tangent route) on the same run."""
    n = 40
    w = small_case(0.8, -2, 1, 170, 26, ext=((15.0, math.pi / 2), (30.0, 1.0)))
    phi0, pi0 = inputs.gaussian_pulse(170, 26, w["rstar_min"], w["rstar_max"], 5.0, 3.0, "regular", 1, -2)
    gser = np.random.default_rng(5).standard_normal((n, 2)) + 1j * np.random.default_rng(6).standard_normal((n, 2))
    out = _run(gpu, w, (phi0, pi0), None, n)
    dlda_fwd = float(np.sum(gser.real * out[5].real + gser.imag * out[5].imag))
    g = _grid(gpu, w)
    g.set_initial_data(torch.from_numpy(phi0).cuda(), torch.from_numpy(pi0).cuda())
    win = g.new_window(n)
    g.step_tangent(n, win)
    lp = torch.zeros((26, 170), dtype=torch.complex128, device="cuda")
    lq = torch.zeros_like(lp)
    dlda_rev = g.adjoint(n, lp, lq, torch.from_numpy(gser).cuda(), win, tangent=True)
    g.close()
    assert abs(dlda_fwd - dlda_rev) <= 1e-10 * abs(dlda_rev), (dlda_fwd, dlda_rev)


def test_full_size_steps(gpu):
    """The adjoint workload's grid (6400 x 256, a = 0.7), two steps from a
    perturbed pulse and a random v, against the oracle."""
    w = inputs.workload("adjoint_a0.7_6400x256")
    phi0, pi0 = inputs.initial_data(w)
    rnd = inputs.random_state(w["nr"], w["ntheta"], seed=17)
    u0 = (phi0 + 1e-3 * rnd[0], pi0 + 1e-3 * rnd[1])
    v0 = inputs.random_state(w["nr"], w["ntheta"], seed=18)
    g = _run(gpu, w, u0, v0, 2)
    o = _oracle(w, u0, v0, 2)
    for k in range(6):
        assert rel_err(g[k], o[k]) <= TOL, k


def test_errors_and_finite_check(gpu):
    w = small_case(0.5, -2, 2, 100, 16)
    g = _grid(gpu, w)
    with pytest.raises(RuntimeError):  # before teuk_enable_adjoint: no a-derivative tables
        ws = torch.empty(gpu.teuk_spin_tangent_workspace_bytes(g.handle) + 256, dtype=torch.uint8, device="cuda")
        gpu.teuk_enable_spin_tangent(g.handle, ws[:gpu.teuk_spin_tangent_workspace_bytes(g.handle)])
    with pytest.raises(RuntimeError):  # not enabled
        gpu.teuk_step_n_spin_tangent(g.handle, 1, None, None)
    u0 = inputs.random_state(100, 16, seed=3)
    u0[0][5, 40] = np.nan
    g.set_initial_data(torch.from_numpy(u0[0]).cuda(), torch.from_numpy(u0[1]).cuda())
    g.set_spin_tangent()
    g.set_finite_check(2)
    with pytest.raises(RuntimeError, match="non-finite"):
        g.step_spin_tangent(5)
    g.close()
