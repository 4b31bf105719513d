"""GPU parity of the forward Lax-Wendroff step (C ABI) against the oracle.

Bar: normwise relative error max|gpu - oracle| / max|oracle| <= 1e-11 on the
state after N steps and on the extraction series (the tolerance named for
this method; both sides compute in IEEE binary64, so the difference is
accumulated rounding of differently ordered but identical arithmetic).
"""
import math

import numpy as np
import pytest

from paper_1010_3816_amd import inputs
from parity import rel_err, run_gpu, run_oracle, small_case

TOL = 1e-11
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("a,s,m,nr,nth", [
    (0.0, -2, 2, 130, 20),     # ragged last strip (130 = 2*62 + 6)
    (0.7, -2, 1, 200, 17),     # odd |m|: anti-mirror ghosts, odd ntheta
    (0.9, 0, -3, 187, 70),     # two theta chunks of 64 plus a tail of 6
    (0.99, -1, 4, 64, 9),
    (0.5, 2, 0, 3, 2),         # smallest grid: one interior column
    (0.3, -2, -2, 63, 2),
])
@pytest.mark.parametrize("block", [None, 0])  # the default (the block pass on grids it takes) and the sweeps
def test_random_state_parity(gpu, a, s, m, nr, nth, block):
    w = small_case(a, s, m, nr, nth)
    phi0, pi0 = inputs.random_state(nr, nth, seed=nr * 131 + nth)
    n = 25
    g = run_gpu(gpu, w, phi0, pi0, n, block_steps=block)
    o = run_oracle(w, phi0, pi0, n)
    assert rel_err(g[0], o[0]) <= TOL
    assert rel_err(g[1], o[1]) <= TOL
    assert rel_err(g[2], o[2]) <= TOL


def test_schwarzschild_400x32_full_run(gpu):
    """The small standard workload, all 1000 steps, at the policy time step.
    Besides its own extraction point (r* = 100, which the pulse does not
    reach within t = 19.6 at that step), a point the pulse does reach
    (about its centre + t/2), so that the series compared is not all tails."""
    w = dict(inputs.workload("schwarzschild_400x32"))
    t_end = w["steps"] * w["dt"]
    w["extract_rstar"] = w["extract_rstar"] + [w["center"] + 0.5 * t_end]
    w["extract_theta"] = w["extract_theta"] + [math.pi / 2]
    phi0, pi0 = inputs.initial_data(w)
    g = run_gpu(gpu, w, phi0, pi0, w["steps"], block_steps=0)  # the sweeps (test_gpu_block: the block pass)
    o = run_oracle(w, phi0, pi0, w["steps"])
    assert np.all(np.isfinite(g[0]))
    assert rel_err(g[0], o[0]) <= TOL
    assert rel_err(g[1], o[1]) <= TOL
    assert rel_err(g[2], o[2]) <= TOL
    assert np.max(np.abs(o[2][:, 1])) > 1e-3 * np.max(np.abs(o[0]))  # a real signal


@pytest.mark.parametrize("tile", [(1, 1), (3, 2), (41, 4), (5, 8), (20, 4)])
def test_tile_shapes_bit_identical(gpu, tile):
    """Every point's arithmetic is independent of the launch shape."""
    w = small_case(0.8, -2, 2, 300, 41, ext=((20.0, 1.0), (-10.0, 2.9), (55.5, 0.01)))
    phi0, pi0 = inputs.random_state(300, 41, seed=5)
    ref = run_gpu(gpu, w, phi0, pi0, 7, tile=(41, 1))
    out = run_gpu(gpu, w, phi0, pi0, 7, tile=tile)
    for k in range(3):
        assert np.array_equal(out[k], ref[k])


@pytest.mark.parametrize("block", [None, 0])  # the block pass (default here) and the sweeps
def test_extraction_points_and_fallback(gpu, block):
    """Poles, grid ends and two points sharing a column (the sweeps: the
    separate-kernel path)."""
    ext = ((20.0, math.pi / 2), (20.0, math.pi / 2 + 0.2), (-30.0, 0.0), (60.0, math.pi), (1.23, 0.05))
    for m in (2, 3):
        w = small_case(0.6, -2, m, 150, 24, ext=ext)
        phi0, pi0 = inputs.random_state(150, 24, seed=m)
        g = run_gpu(gpu, w, phi0, pi0, 9, block_steps=block)
        o = run_oracle(w, phi0, pi0, 9)
        assert g[2].shape == (9, len(ext))
        assert rel_err(g[2], o[2]) <= TOL


def test_user_coefficients_dalembert(gpu):
    """USER mode with the d'Alembert coefficients: exact translation at Courant 1."""
    nr, nth = 200, 4
    w = dict(a=0.0, s=0, m=0, nr=nr, ntheta=nth, rstar_min=-10.0, rstar_max=10.0)
    w["dt"] = (w["rstar_max"] - w["rstar_min"]) / (nr - 1)
    ci = np.zeros((9, nth, nr))
    ch = np.zeros((9, nth, nr - 1))
    ci[0] = 1.0
    ch[0] = 1.0
    x = np.linspace(-10.0, 10.0, nr)
    phi0 = np.tile(np.exp(-((x + 4.0) ** 2)) * (1 + 0.3j), (nth, 1))
    pi0 = np.zeros_like(phi0)
    g = run_gpu(gpu, w, phi0, pi0, 40, coef=(ci, ch))
    o = run_oracle(w, phi0, pi0, 40, coef=(ci, ch))
    assert rel_err(g[0], o[0]) <= TOL
    p0 = phi0.copy()
    p0[:, 0] = p0[:, -1] = 0
    expect = np.zeros_like(p0)
    expect[:, 41:nr - 1] = p0[:, 1:nr - 41]
    assert np.max(np.abs(g[0] - expect)) < 1e-14


def test_user_coefficients_random(gpu):
    """USER mode with arbitrary 2-D coefficient tables."""
    nr, nth = 90, 13
    rng = np.random.default_rng(11)
    ci = rng.uniform(-0.5, 0.5, (9, nth, nr))
    ch = rng.uniform(-0.5, 0.5, (9, nth, nr - 1))
    ci[0] += 1.0
    ch[0] += 1.0
    w = dict(a=0.0, s=0, m=1, nr=nr, ntheta=nth, rstar_min=0.0, rstar_max=30.0, dt=0.01,
             extract_rstar=[12.3], extract_theta=[0.7])
    phi0, pi0 = inputs.random_state(nr, nth, seed=4)
    g = run_gpu(gpu, w, phi0, pi0, 12, coef=(ci, ch))
    o = run_oracle(w, phi0, pi0, 12, coef=(ci, ch))
    assert rel_err(g[0], o[0]) <= TOL
    assert rel_err(g[1], o[1]) <= TOL
    assert rel_err(g[2], o[2]) <= TOL


@pytest.mark.parametrize("name,steps", [("kerr_a0.9_6400x256", 3), ("kerr_a0.99_25600x512", 2)])
def test_full_size_workloads(gpu, name, steps):
    """Full-size grids in the default launch configuration: the whole state
    after a few steps against the oracle."""
    w = inputs.workload(name)
    phi0, pi0 = inputs.initial_data(w)
    rnd = inputs.random_state(w["nr"], w["ntheta"], seed=3)
    phi0 = phi0 + 1e-3 * rnd[0]
    pi0 = pi0 + 1e-3 * rnd[1]
    g = run_gpu(gpu, w, phi0, pi0, steps)
    o = run_oracle(w, phi0, pi0, steps)
    assert rel_err(g[0], o[0]) <= TOL
    assert rel_err(g[1], o[1]) <= TOL
    if g[2] is not None:
        assert rel_err(g[2], o[2]) <= TOL


def test_state_round_trip_and_finite_check(gpu):
    import torch

    w = small_case(0.4, 0, 1, 77, 6)
    phi0, pi0 = inputs.random_state(77, 6, seed=9)
    g = gpu.TeukGrid(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["dt"])
    g.set_initial_data(torch.from_numpy(phi0).cuda(), torch.from_numpy(pi0).cuda())
    p, q = g.state()
    exp_p, exp_q = phi0.copy(), pi0.copy()
    for arr in (exp_p, exp_q):
        arr[:, 0] = 0
        arr[:, -1] = 0
    assert np.array_equal(p.cpu().numpy(), exp_p) and np.array_equal(q.cpu().numpy(), exp_q)
    assert g.check_finite()
    assert g.steps == 0
    g.step(3)
    assert g.steps == 3
    bad = phi0.copy()
    bad[3, 40] = np.nan
    g.set_initial_data(torch.from_numpy(bad).cuda(), torch.from_numpy(pi0).cuda())
    assert not g.check_finite()
    g.close()


@pytest.mark.parametrize("block", [None, 0])  # the default (the block pass here) and the sweeps
def test_step_split_invariance_and_zero_steps(gpu, block):
    """n steps in one call equal the same steps split over several calls, bit
    for bit, series included (the sample of each call's first input state is
    fused into the next kernel, the last one taken after the loop); a call
    with n = 0 changes nothing."""
    import torch

    w = small_case(0.9, -2, 3, 211, 37, ext=((20.0, math.pi / 2), (-12.0, 0.3)))
    phi0, pi0 = inputs.random_state(211, 37, seed=17)
    ref = run_gpu(gpu, w, phi0, pi0, 12, block_steps=block)
    g = gpu.TeukGrid(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["dt"],
                     extract_rstar=w["extract_rstar"], extract_theta=w["extract_theta"])
    if block is not None:
        g.set_block_steps(block)
    g.set_initial_data(torch.from_numpy(phi0).cuda(), torch.from_numpy(pi0).cuda())
    parts = []
    for n in (1, 0, 5, 6):
        s = g.step(n)
        if n == 0:
            assert s is None and g.steps == 1
        else:
            parts.append(s.cpu().numpy())
    phi, pi = (t.cpu().numpy() for t in g.state())
    assert g.steps == 12
    assert np.array_equal(phi, ref[0]) and np.array_equal(pi, ref[1])
    assert np.array_equal(np.concatenate(parts), ref[2])
    g.close()


@pytest.mark.parametrize("a,s,m,nr,nth,n,tile", [
    (0.7, -2, 2, 130, 20, 9, (16, 4)),   # ragged strips (130 = 2*60 + 10), odd n: a single last step
    (0.9, 0, -3, 187, 70, 8, (16, 4)),   # odd |m|, five chunks with a ragged last one
    (0.99, -1, 4, 64, 9, 6, (3, 2)),     # three-row chunks: halo rows from two chunks away
    (0.5, 2, 0, 3, 2, 5, (1, 1)),        # smallest grid, one-row chunks
    (0.3, -2, -2, 63, 2, 4, (2, 4)),     # both rows are pole rows
    (0.8, -2, 1, 300, 41, 10, (41, 8)),  # one chunk; eight waves requested, four used
    # at least 64 strips: tiles in runs of strips per XCD, uneven runs
    (0.7, -2, 2, 3845, 12, 5, (5, 4)),   # 65 strips (runs of 8 and one of 9), chunks of 5, 5, 2
    (0.9, 0, -3, 4323, 7, 4, (3, 1)),    # 73 strips, one wave per workgroup, chunks of 3, 3, 1
])
def test_two_step_passes_bit_identical(gpu, a, s, m, nr, nth, n, tile):
    """Two steps per pass (temporal blocking) give exactly the single-step
    results, state and extraction series included."""
    w = small_case(a, s, m, nr, nth, ext=((20.0, math.pi / 2), (-12.0, 0.3)))
    phi0, pi0 = inputs.random_state(nr, nth, seed=nr * 7 + nth)
    one = run_gpu(gpu, w, phi0, pi0, n, tile=tile, steps_per_pass=1)
    two = run_gpu(gpu, w, phi0, pi0, n, tile=tile, steps_per_pass=2)
    for k in range(3):
        assert np.array_equal(two[k], one[k]), k
    o = run_oracle(w, phi0, pi0, n)
    assert rel_err(two[0], o[0]) <= TOL
    assert rel_err(two[2], o[2]) <= TOL


@pytest.mark.parametrize("spp", [1, 2])
def test_cache_policies_bit_identical(gpu, spp):
    """Cache-keeping and streaming stores of the next state give the same
    results bit for bit, and the default policy keeps the states of a grid
    whose two states fit in 192 MiB and streams those of a larger one."""
    w = small_case(0.7, -2, 2, 190, 30, ext=((20.0, math.pi / 2),))
    phi0, pi0 = inputs.random_state(190, 30, seed=97)
    keep = run_gpu(gpu, w, phi0, pi0, 9, steps_per_pass=spp, cache_policy=gpu.TEUK_CACHE_KEEP)
    stream = run_gpu(gpu, w, phi0, pi0, 9, steps_per_pass=spp, cache_policy=gpu.TEUK_CACHE_STREAM)
    auto = run_gpu(gpu, w, phi0, pi0, 9, steps_per_pass=spp)
    for k in range(3):
        assert np.array_equal(keep[k], stream[k]) and np.array_equal(auto[k], keep[k]), k
    for (nr, nth), kept in (((6400, 256), True), ((6400, 512), False)):
        g = gpu.TeukGrid(0.5, -2, 2, nr, nth, -100.0, 600.0, 0.01)
        assert g.cache_policy() == (gpu.TEUK_CACHE_AUTO, kept)
        g.set_cache_policy(gpu.TEUK_CACHE_KEEP)
        assert g.cache_policy() == (gpu.TEUK_CACHE_KEEP, True)
        with pytest.raises(RuntimeError):
            g.set_cache_policy(3)
        g.close()


def test_two_step_extraction_fallback(gpu):
    """Two extraction points in one two-step tile: the pairs of steps fall
    back to single steps with the separate extraction pass."""
    w = small_case(0.6, -2, 2, 150, 24, ext=((20.0, math.pi / 2), (20.5, math.pi / 2 + 0.1), (-3.0, 1.0)))
    phi0, pi0 = inputs.random_state(150, 24, seed=23)
    one = run_gpu(gpu, w, phi0, pi0, 7, steps_per_pass=1)
    two = run_gpu(gpu, w, phi0, pi0, 7, steps_per_pass=2)
    for k in range(3):
        assert np.array_equal(two[k], one[k]), k


@pytest.mark.parametrize("name", ["kerr_a0.9_6400x256", "kerr_a0.99_25600x512"])
def test_two_step_full_size(gpu, name):
    """Full-size grids, two steps per pass, against the oracle."""
    w = inputs.workload(name)
    phi0, pi0 = inputs.initial_data(w)
    rnd = inputs.random_state(w["nr"], w["ntheta"], seed=13)
    phi0 = phi0 + 1e-3 * rnd[0]
    pi0 = pi0 + 1e-3 * rnd[1]
    g = run_gpu(gpu, w, phi0, pi0, 2, steps_per_pass=2)
    o = run_oracle(w, phi0, pi0, 2)
    assert rel_err(g[0], o[0]) <= TOL
    assert rel_err(g[1], o[1]) <= TOL
    if g[2] is not None:
        assert rel_err(g[2], o[2]) <= TOL


@pytest.mark.parametrize("name", ["kerr_a0.9_6400x256", "kerr_a0.99_25600x512"])
def test_full_length_run(gpu, name):
    """The whole run of a full-size workload (all its steps, from its own
    initial data) in the default launch configuration: one and two steps per
    pass agree bit for bit in the final state and the whole extraction
    series, and the last step equals one oracle step taken from the GPU's
    own state before it."""
    import torch

    import oracle

    w = inputs.workload(name)
    n = w["steps"]
    phi0, pi0 = inputs.initial_data(w)
    runs = {}
    for spp in (2, 1):
        g = gpu.TeukGrid(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["dt"],
                         extract_rstar=w.get("extract_rstar", []), extract_theta=w.get("extract_theta", []))
        g.set_steps_per_pass(spp)
        g.set_initial_data(torch.from_numpy(phi0).cuda(), torch.from_numpy(pi0).cuda())
        s1 = g.step(n - 1)
        before = [t.cpu().numpy() for t in g.state()]
        s2 = g.step(1)
        after = [t.cpu().numpy() for t in g.state()]
        series = None if s1 is None else np.concatenate([s1.cpu().numpy(), s2.cpu().numpy()])
        runs[spp] = (before, after, series)
        g.close()
    for k in range(2):
        assert np.array_equal(runs[1][1][k], runs[2][1][k]), k
    if runs[2][2] is not None:
        assert runs[2][2].shape == (n, len(w["extract_rstar"]))
        assert np.array_equal(runs[1][2], runs[2][2])
        assert np.isfinite(runs[2][2]).all()
    before, after = runs[2][0], runs[2][1]
    assert np.isfinite(after[0]).all() and np.isfinite(after[1]).all()
    o = oracle.OracleGrid(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["dt"])
    p, q = o.step(before[0], before[1], 1)
    assert rel_err(after[0], p) <= TOL
    assert rel_err(after[1], q) <= TOL


def _default_rows(nr, nth, cus):
    """The documented default tile height: fewest rounds k of two wavefronts
    per SIMD whose round-filling tiles have at most 64 rows."""
    strips = -(-nr // 60)
    r = 64
    for k in range(1, 65):
        chunks = k * cus * 8 // strips
        if chunks >= 1 and -(-nth // chunks) <= 64:
            r = -(-nth // chunks)
            break
    return min(r, nth)


def _default_adjoint_rows(nr, nth, cus):
    chunks = cus * 7 // -(-nr // 62)
    if chunks < 1:
        return min(nth, 16)
    return min(-(-nth // chunks), 16, nth)


@pytest.mark.parametrize("nr,nth", [(25600, 512), (6400, 256), (400, 32), (12800, 128), (70000, 64)])
def test_default_tile_fills_whole_rounds(gpu, nr, nth):
    import torch

    cus = torch.cuda.get_device_properties(0).multi_processor_count
    w = small_case(0.5, -2, 2, nr, nth)
    g = gpu.TeukGrid(w["a"], w["s"], w["m"], nr, nth, w["rstar_min"], w["rstar_max"], w["dt"])
    rows, wpb = g.tile()
    adj = g.adjoint_tile()
    g.close()
    assert rows == _default_rows(nr, nth, cus)
    tiles = -(-nr // 60) * -(-nth // rows)
    assert wpb == (1 if tiles < 4 * cus else 4)
    assert adj == (_default_adjoint_rows(nr, nth, cus), 4)
    if cus == 256:
        expect = {(25600, 512): (57, 4, 16), (6400, 256): (14, 4, 16), (400, 32): (1, 1, 1)}.get((nr, nth))
        if expect:
            assert (rows, wpb, adj[0]) == expect


def test_full_size_tile_independence(gpu):
    """Every launch shape the benchmark's autotuner may pick gives the same
    state, bit for bit, on the full 25600 x 512 grid (the default shape is
    checked against the oracle in test_two_step_full_size)."""
    import torch

    from paper_1010_3816_amd import autotune

    w = inputs.workload("kerr_a0.99_25600x512")
    phi0, pi0 = inputs.initial_data(w)
    rnd = inputs.random_state(w["nr"], w["ntheta"], seed=17)
    phi0 = phi0 + 1e-3 * rnd[0]
    pi0 = pi0 + 1e-3 * rnd[1]
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    g = gpu.TeukGrid(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["dt"])
    P0 = torch.from_numpy(phi0).cuda()
    Q0 = torch.from_numpy(pi0).cuda()
    g.set_initial_data(P0, Q0)
    g.step(3)
    ref = [t.clone() for t in g.state()]
    rows = sorted(set(autotune.GRID_ROWS) | set(autotune.round_rows(w["nr"], w["ntheta"], cus)))
    for r in rows:
        for wpb in (1, 2, 4):
            g.set_tile(r, wpb)
            g.set_initial_data(P0, Q0)
            g.step(3)
            p, q = g.state()
            assert torch.equal(p, ref[0]) and torch.equal(q, ref[1]), (r, wpb)
    g.close()


def test_policy_time_step(gpu):
    """dt <= 0 takes the policy step (teuk_suggest_dt with a growth bound of
    10 over stable_steps steps, 10,000 by default, Courant 0.5), reported by
    teuk_get_dt and used by the steps (parity with the oracle at that dt);
    strict mode accepts a dt below its bound."""
    import torch

    from paper_1010_3816_amd import binding

    w = small_case(0.7, -2, 2, 150, 20)
    geo = (w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"])
    for horizon, n_pol in ((0, 10000), (200, 200)):
        g = gpu.TeukGrid(*geo, 0.0, extract_rstar=w["extract_rstar"], extract_theta=w["extract_theta"],
                         stable_steps=horizon)
        dt = g.dt
        assert dt == binding.suggest_dt(*geo, n_pol, 10.0, 0.5)
        phi0, pi0 = inputs.random_state(w["nr"], w["ntheta"], seed=21)
        g.set_initial_data(torch.from_numpy(phi0).cuda(), torch.from_numpy(pi0).cuda())
        ser = g.step(9).cpu().numpy()
        got = [t.cpu().numpy() for t in g.state()]
        g.close()
        o = run_oracle(dict(w, dt=dt), phi0, pi0, 9)
        assert rel_err(got[0], o[0]) <= TOL and rel_err(got[1], o[1]) <= TOL and rel_err(ser, o[2]) <= TOL
    ok = 0.99 * binding.suggest_dt(*geo, 500, 10.0, 1.0)
    g = gpu.TeukGrid(*geo, ok, stable_steps=500)
    assert g.dt == ok
    g.close()


def test_maximum_sizes(gpu):
    """The largest grids the ABI accepts, one in each direction, a few steps
    with one and two steps per pass (bit-identical).  Nr = 2^24 x Ntheta = 2
    (both rows are pole rows): the oracle on windows of 2000 columns at both
    radial ends and in the middle, compared where the window's own edges
    (zeroed like radial boundaries) cannot have reached in n steps (one
    column per step).  Nr = 3 x Ntheta = 2^20: the whole grid."""
    import torch

    import oracle

    n = 3
    for nr, nth in ((1 << 24, 2), (3, 1 << 20)):
        w = small_case(0.6, -2, 1, nr, nth, rmin=-50.0, rmax=150.0, ext=())
        phi0, pi0 = inputs.random_state(nr, nth, seed=31)
        g = gpu.TeukGrid(w["a"], w["s"], w["m"], nr, nth, w["rstar_min"], w["rstar_max"], w["dt"])
        states = []
        for spp in (2, 1):
            g.set_steps_per_pass(spp)
            g.set_initial_data(torch.from_numpy(phi0).cuda(), torch.from_numpy(pi0).cuda())
            g.step(n)
            states.append([t.cpu().numpy() for t in g.state()])
        assert g.check_finite()
        g.close()
        for k in range(2):
            assert np.array_equal(states[0][k], states[1][k]), (nr, nth, k)
        got = states[0]
        if nr == 3:
            o = run_oracle(w, phi0, pi0, n)
            assert rel_err(got[0], o[0]) <= TOL and rel_err(got[1], o[1]) <= TOL
            continue
        dr = (w["rstar_max"] - w["rstar_min"]) / (nr - 1)
        for i0 in (0, nr // 2 - 1000, nr - 2000):
            i1 = i0 + 1999
            o = oracle.OracleGrid(w["a"], w["s"], w["m"], 2000, nth, w["rstar_min"] + i0 * dr,
                                  w["rstar_min"] + i1 * dr, w["dt"])
            p, q = o.project(phi0[:, i0:i1 + 1], pi0[:, i0:i1 + 1])
            p, q, _ = o.evolve(p, q, n, [], [])
            lo = 0 if i0 == 0 else n + 1  # columns the window's artificial edges cannot have reached
            hi = 2000 if i1 == nr - 1 else 2000 - n - 1
            for a, b in ((got[0][:, i0:i1 + 1], p), (got[1][:, i0:i1 + 1], q)):
                assert rel_err(a[:, lo:hi], b[:, lo:hi]) <= TOL, (i0, rel_err(a[:, lo:hi], b[:, lo:hi]))


def test_in_loop_finite_check(gpu):
    """teuk_set_finite_check: a NaN planted in the initial data is reported by
    the first check (after `every` steps); a run at the literal time step
    0.5 dr* of the 400 x 32 grid, which blows up, is reported by the first
    check at or after the step at which the oracle's state first turns
    non-finite; a finite run returns normally; the checked calls take all
    their steps, with the states of unchecked calls."""
    import torch

    import oracle

    w = small_case(0.5, -2, 2, 150, 24, ext=())
    phi0, pi0 = inputs.random_state(150, 24, seed=3)
    bad = phi0.copy()
    bad[7, 40] = np.nan
    g = gpu.TeukGrid(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["dt"])
    g.set_block_steps(0)  # the sweeps' check points (test_gpu_block: the block pass's)
    g.set_finite_check(10)
    g.set_initial_data(torch.from_numpy(bad).cuda(), torch.from_numpy(pi0).cuda())
    with pytest.raises(gpu.TeukError) as ei:
        g.step(25)
    assert ei.value.code == gpu.TEUK_E_NONFINITE and "after step 10" in str(ei.value), str(ei.value)
    assert g.steps == 25
    g.set_initial_data(torch.from_numpy(phi0).cuda(), torch.from_numpy(pi0).cuda())
    g.step(25)  # finite: no error, and the flag of the failed call was cleared
    checked = [t.cpu().numpy() for t in g.state()]
    g.close()
    ref = run_gpu(gpu, w, phi0, pi0, 25, block_steps=0)
    assert np.array_equal(checked[0], ref[0]) and np.array_equal(checked[1], ref[1])

    # blow-up at the literal time step
    wl = dict(inputs.workload("schwarzschild_400x32"))
    wl["dt"] = 0.5 * (wl["rstar_max"] - wl["rstar_min"]) / (wl["nr"] - 1)
    p0, q0 = inputs.initial_data(wl)
    o = oracle.OracleGrid(wl["a"], wl["s"], wl["m"], wl["nr"], wl["ntheta"], wl["rstar_min"], wl["rstar_max"],
                          wl["dt"])
    p, q = o.project(p0, q0)
    first = None
    for k in range(1, 1001):
        p, q = o.step(p, q, 1)
        if not (np.isfinite(p).all() and np.isfinite(q).all()):
            first = k
            break
    assert first is not None and first > 20
    every = 7
    g = gpu.TeukGrid(wl["a"], wl["s"], wl["m"], wl["nr"], wl["ntheta"], wl["rstar_min"], wl["rstar_max"], wl["dt"])
    g.set_block_steps(0)
    g.set_finite_check(every)
    g.set_initial_data(torch.from_numpy(p0).cuda(), torch.from_numpy(q0).cuda())
    with pytest.raises(gpu.TeukError) as ei:
        g.step(first + 100)
    assert ei.value.code == gpu.TEUK_E_NONFINITE
    seen = int(str(ei.value).rsplit("after step ", 1)[1].split()[0])
    # checks run at the first pass boundary (two steps per pass) at or after each multiple of `every`
    assert first - 1 <= seen <= first + every + 2, (first, seen)
    g.close()
