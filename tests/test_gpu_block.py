"""The small-grid block pass (teuk_set_block_launch) through the C ABI.

The pass keeps a workgroup's columns by all theta rows of the state in LDS
and takes several steps per launch; its per-point arithmetic is that of the
sweeps (Sec. 3.2, Eqs. (lw1)-(lw2)), so the state and the extraction series
must equal the two-step sweeps' bit for bit, and the oracle's within the
forward bar (normwise 1e-11).
"""
import math

import numpy as np
import pytest
import torch

from paper_1010_3816_amd import inputs
from parity import rel_err, run_gpu, run_oracle, small_case

TOL = 1e-11
pytestmark = pytest.mark.gpu


def _max_cols(nth):
    """The most columns a workgroup may hold (1024 threads, 64 columns)."""
    return min(64, 1024 // nth)


@pytest.mark.parametrize("a,s,m,nr,nth,n,k,c,ext", [
    # 400 x 32 with 32 columns a workgroup, 8 steps a launch, 37 steps: the
    # extraction point of that workload and one at the last written column
    # of the first workgroup (its right neighbour is a halo column there)
    (0.0, -2, 2, 400, 32, 37, 8, 32, ((20.0, math.pi / 2), (-50.0 + 15.4 * 200.0 / 399, 1.0))),
    (0.0, -2, 2, 400, 32, 20, 15, 32, ((20.0, math.pi / 2),)),  # the most steps a launch for 32 columns
    (0.0, -2, 2, 400, 32, 23, 7, 16, ((-50.0 + 1.5 * 200.0 / 399, 0.7),)),  # 16 columns (the default there)
    (0.4, -2, 2, 100, 32, 8, 3, 8, ((5.0, 1.1),)),             # 8 columns: 2 written a workgroup
    (0.6, 1, -1, 200, 20, 9, 4, 25, ((11.0, 0.4),)),           # an odd width
    (0.3, -2, -2, 63, 2, 11, 5, 64, ((10.0, 0.2),)),           # two rows, both pole rows
    (0.9, 0, -3, 150, 64, 9, 7, 16, ((20.0, 2.9), (-5.0, 0.01))),  # 64 rows, 7 steps; odd m; pole points
    (0.7, -1, 1, 130, 7, 10, 3, 64, ((20.0, 1.0), (21.0, 1.2))),  # odd row count, two points in one workgroup
    (0.5, 2, 0, 3, 5, 6, 2, 64, ()),                           # three columns, one workgroup
    (0.99, -2, 4, 257, 30, 13, 1, 34, ((0.0, 0.5),)),          # one step a launch
])
def test_block_pass_bit_identical(gpu, a, s, m, nr, nth, n, k, c, ext):
    """Launches of k steps over c-column workgroups give exactly the sweeps'
    state and series."""
    rmin, rmax = (-50.0, 150.0) if nr == 400 else (-30.0, 60.0)
    w = small_case(a, s, m, nr, nth, rmin=rmin, rmax=rmax, ext=ext)
    phi0, pi0 = inputs.random_state(nr, nth, seed=nr * 13 + nth + k)
    ref = run_gpu(gpu, w, phi0, pi0, n, block_steps=0)
    blk = run_gpu(gpu, w, phi0, pi0, n, block_steps=k, block_cols=c)
    for i in range(3):
        if ref[i] is None:
            assert blk[i] is None
        else:
            assert np.array_equal(blk[i], ref[i]), i
    o = run_oracle(w, phi0, pi0, n)
    assert rel_err(blk[0], o[0]) <= TOL
    assert rel_err(blk[1], o[1]) <= TOL
    if o[2] is not None and o[2].size:
        assert rel_err(blk[2], o[2]) <= TOL


@pytest.mark.parametrize("case", range(10))
def test_block_pass_random_configs(gpu, case):
    """Seeded random grids (ntheta <= 64), spins, modes, workgroup widths,
    steps per launch, step counts and extraction points: the sweeps' results
    bit for bit, the oracle's within the bar."""
    rng = np.random.default_rng(4200 + case)
    nth = int(rng.integers(2, 65))
    nr = int(rng.integers(3, 500))
    c = int(rng.integers(4, _max_cols(nth) + 1))
    k = int(rng.integers(1, (c - 2) // 2 + 1))
    n = int(rng.integers(1, 3 * k + 3))
    n_ext = int(rng.integers(0, 9))
    ext = tuple((float(rng.uniform(-30.0, 60.0)), float(rng.uniform(0.0, math.pi))) for _ in range(n_ext))
    w = small_case(float(rng.uniform(0.0, 0.99)), int(rng.choice([-2, -1, 0, 1, 2])), int(rng.integers(-4, 5)),
                   nr, nth, ext=ext)
    phi0, pi0 = inputs.random_state(nr, nth, seed=4300 + case)
    ref = run_gpu(gpu, w, phi0, pi0, n, block_steps=0)
    blk = run_gpu(gpu, w, phi0, pi0, n, block_steps=k, block_cols=c)
    for i in range(3):
        if ref[i] is None:
            assert blk[i] is None
        else:
            assert np.array_equal(blk[i], ref[i]), (case, nr, nth, c, k, n, i)
    o = run_oracle(w, phi0, pi0, n)
    assert rel_err(blk[0], o[0]) <= TOL and rel_err(blk[1], o[1]) <= TOL, (case, nr, nth, c, k, n)


def test_block_pass_many_points_falls_back(gpu):
    """More than 8 extraction points: teuk_step_n keeps the sweeps for a
    series (same results), and takes the block pass without one."""
    ext = tuple((-20.0 + 7.0 * i, 0.3 + 0.25 * i) for i in range(9))
    w = small_case(0.6, -2, 2, 200, 16, ext=ext)
    phi0, pi0 = inputs.random_state(200, 16, seed=5)
    ref = run_gpu(gpu, w, phi0, pi0, 9, block_steps=0)
    blk = run_gpu(gpu, w, phi0, pi0, 9, block_steps=6, block_cols=32)
    for i in range(3):
        assert np.array_equal(blk[i], ref[i]), i
    g = gpu.TeukGrid(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["dt"],
                     extract_rstar=w["extract_rstar"], extract_theta=w["extract_theta"])
    g.set_block_launch(6, 32)
    g.set_initial_data(torch.from_numpy(phi0).cuda(), torch.from_numpy(pi0).cuda())
    assert g.step(9, series=False) is None
    phi, pi = (t.cpu().numpy() for t in g.state())
    assert np.array_equal(phi, ref[0]) and np.array_equal(pi, ref[1])
    g.close()


def _default_launch(nr, nth, cus):
    """The library's default: over workgroups of up to 256, 512 and 1024
    threads, the most steps (at least 4) whose workgroups fit one per CU,
    scored 0.8 ns per point a workgroup holds + 3.6 us / steps; (0, 0) when
    none fits."""
    if nth > 64:
        return 0, 0
    best = None
    for threads in (256, 512, 1024):
        c = min(64, threads // nth)
        for k in range((c - 2) // 2, 3, -1):
            if -(-nr // (c - 2 * k)) <= cus:
                score = 0.8e-3 * c * nth + 3.6 / k
                if best is None or score < best[0]:
                    best = (score, k, c)
                break
    return (0, 0) if best is None else best[1:]


def test_block_launch_default(gpu):
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    for nr, nth in ((400, 32), (800, 32), (3200, 32), (1600, 64), (6400, 64), (400, 16), (400, 65), (25600, 16),
                    (3, 2)):
        g = gpu.TeukGrid(0.5, -2, 2, nr, nth, -50.0, 150.0, 0.001)
        assert g.block_launch() == _default_launch(nr, nth, cus), (nr, nth, cus)
        g.close()
    if cus == 256:  # the device these widths were measured on
        assert _default_launch(400, 32, cus) == (7, 16) and _default_launch(400, 16, cus) == (15, 32)
        assert _default_launch(3200, 32, cus) == (9, 32) and _default_launch(6400, 64, cus) == (0, 0)


def test_block_pass_full_run_against_oracle(gpu):
    """The 400 x 32 workload over all its 1000 steps with the default launch
    (the block pass), against the oracle, with a point the pulse reaches."""
    w = dict(inputs.workload("schwarzschild_400x32"))
    assert _default_launch(400, 32, torch.cuda.get_device_properties(0).multi_processor_count)[0] > 0
    n = w["steps"]
    t_end = n * w["dt"]
    w["extract_rstar"] = w["extract_rstar"] + [w["center"] + 0.5 * t_end]
    w["extract_theta"] = w["extract_theta"] + [math.pi / 2]
    phi0, pi0 = inputs.initial_data(w)
    g = run_gpu(gpu, w, phi0, pi0, n)
    o = run_oracle(w, phi0, pi0, n)
    assert rel_err(g[0], o[0]) <= TOL
    assert rel_err(g[1], o[1]) <= TOL
    assert rel_err(g[2], o[2]) <= TOL
    assert np.max(np.abs(o[2][:, 1])) > 1e-3 * np.max(np.abs(o[0]))  # a real signal


def test_block_launch_api(gpu):
    """Range checks: 4 <= cols <= min(64, 1024 / ntheta), 0 <= steps <=
    (cols - 2) / 2, cols 0 keeps the grid's; no block pass for ntheta > 64 or
    user coefficients."""
    g = gpu.TeukGrid(0.5, -2, 2, 400, 32, -50.0, 150.0, 0.01)
    g.set_block_launch(15, 32)
    assert g.block_launch() == (15, 32)
    g.set_block_launch(3, 8)
    assert g.block_launch() == (3, 8)
    g.set_block_launch(2)  # cols 0: keeps 8
    assert g.block_launch() == (2, 8)
    for bad in ((-1, 32), (16, 32), (4, 8), (1, 3), (1, 33), (1, 65)):
        with pytest.raises(RuntimeError):
            g.set_block_launch(*bad)
    assert g.block_launch() == (2, 8)
    g.set_block_launch(0)
    assert g.block_steps() == 0
    g.close()
    g = gpu.TeukGrid(0.5, -2, 2, 400, 65, -50.0, 150.0, 0.01)
    assert g.block_launch() == (0, 0)
    with pytest.raises(RuntimeError):
        g.set_block_launch(1, 8)
    g.set_block_launch(0)
    g.close()
    g = gpu.TeukGrid(0.5, -2, 2, 50, 8, -50.0, 150.0, 0.01, coef_mode=gpu.TEUK_COEF_USER)
    with pytest.raises(RuntimeError):
        g.set_block_launch(2, 16)
    g.close()


def test_block_pass_finite_check(gpu):
    """The in-loop finite check sees a state the block pass made non-finite:
    launches of 5 steps, a check every 10 steps, reported after step 10."""
    w = small_case(0.5, -2, 2, 120, 16, ext=())
    phi0, pi0 = inputs.random_state(120, 16, seed=11)
    phi0[3, 40] = np.nan
    g = gpu.TeukGrid(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["dt"])
    g.set_block_launch(5, 32)
    g.set_finite_check(10)
    g.set_initial_data(torch.from_numpy(phi0).cuda(), torch.from_numpy(pi0).cuda())
    with pytest.raises(gpu.TeukError) as ei:
        g.step(24)
    assert ei.value.code == gpu.TEUK_E_NONFINITE and "after step 10" in str(ei.value), str(ei.value)
    assert g.steps == 24
    g.close()


@pytest.mark.parametrize("k,c", [(5, 16), (7, 32), (2, 8)])
def test_block_pass_points_sharing_rows(gpu, k, c):
    """Points whose samples fall on the same thread: at one r*, point A on
    rows 3, 4 and point B on rows 4, 5 (the thread of row 4 samples for
    both), a copy of A (two samples of one row in one step), and a point in
    the first column of a workgroup; the sweeps' series bit for bit."""
    nth = 16
    dth = math.pi / nth
    ra = -30.0 + 37.3 * 90.0 / 199
    ext = ((ra, 3.8 * dth), (ra, 5.1 * dth), (ra, 3.8 * dth), (-30.0 + (c - 2 * k) * 90.0 / 199, 0.9))
    w = small_case(0.6, -2, 2, 200, nth, rmin=-30.0, rmax=60.0, ext=ext)
    phi0, pi0 = inputs.random_state(200, nth, seed=700 + c)
    n = 3 * k + 1
    ref = run_gpu(gpu, w, phi0, pi0, n, block_steps=0)
    blk = run_gpu(gpu, w, phi0, pi0, n, block_steps=k, block_cols=c)
    for i in range(3):
        assert np.array_equal(blk[i], ref[i]), i
    assert np.array_equal(blk[2][:, 0], blk[2][:, 2])  # the copy of A
    o = run_oracle(w, phi0, pi0, n)
    assert rel_err(blk[2], o[2]) <= TOL
