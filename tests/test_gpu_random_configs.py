"""Seeded random configurations through the C ABI against the oracle.

Each case draws the grid size (Nr in [3, 700), Ntheta in [2, 80)), the spin,
the spin weight, the mode, the launch shape, the number of steps and up to
three extraction points from a fixed-seed generator, so that the sweep covers
combinations the hand-written cases do not (ragged strips and chunks of every
size, pole rows inside and at the edges of tiles, extraction points anywhere).

Forward: one and two steps per pass bit-identical; state and series within
1e-11 normwise of the oracle; a longer run with the in-loop finite check on
(random interval) bit-identical to one without it.  Adjoint: the spin path's
cotangents within 1e-11 of the oracle's transposed steps and dL/da within
1e-10; the cotangent-only paths (one and two steps per pass) and the
stored-tangent route bit-identical to the spin path's cotangents, the
tangent route's dL/da within 1e-10 of the oracle.  Spin derivative carried
forward: u, v and both sample series within 1e-11 of the oracle's forward-mode
evolution from random u and v, u and its series bit-identical to the forward
path.  Batch: random member sets
and persistent launch shapes bit-identical to single-grid evolutions and
extractions.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1010_3816_amd import inputs
from parity import oracle_segment_adjoint, rel_err, run_gpu, run_oracle, small_case

pytestmark = pytest.mark.gpu
TOL = 1e-11


def _draw(seed, n_max, ext_min):
    rng = np.random.default_rng(seed)
    c = dict(nr=int(rng.integers(3, 700)), nth=int(rng.integers(2, 80)), a=float(rng.uniform(0, 0.99)),
             s=int(rng.choice([-2, -1, 0, 1, 2])), m=int(rng.integers(-4, 5)))
    c["rows"] = int(rng.integers(1, c["nth"] + 1))
    c["wpb"] = int(rng.choice([1, 2, 4]))
    c["n"] = int(rng.integers(1, n_max))
    ne = int(rng.integers(ext_min, 4))
    c["ext"] = tuple((float(rng.uniform(-30.0, 60.0)), float(rng.uniform(0, math.pi))) for _ in range(ne))
    c["gser"] = rng.standard_normal((c["n"], max(ne, 1))) + 1j * rng.standard_normal((c["n"], max(ne, 1)))
    c["long_n"] = int(rng.integers(4, 24))  # drawn last: the earlier draws are unchanged
    c["check_every"] = int(rng.integers(1, 6))
    return c


@pytest.mark.parametrize("case", range(24))
def test_random_forward(gpu, case):
    c = _draw(5000 + case, 10, 0)
    w = small_case(c["a"], c["s"], c["m"], c["nr"], c["nth"], ext=c["ext"])
    phi0, pi0 = inputs.random_state(c["nr"], c["nth"], seed=6000 + case)
    one = run_gpu(gpu, w, phi0, pi0, c["n"], tile=(c["rows"], c["wpb"]), steps_per_pass=1)
    two = run_gpu(gpu, w, phi0, pi0, c["n"], tile=(c["rows"], c["wpb"]), steps_per_pass=2)
    for k in range(3):
        if one[k] is not None:
            assert np.array_equal(one[k], two[k]), (c, k)
    o = run_oracle(w, phi0, pi0, c["n"])
    assert rel_err(two[0], o[0]) <= TOL and rel_err(two[1], o[1]) <= TOL, c
    if c["ext"]:
        assert rel_err(two[2], o[2]) <= TOL, c
    # a longer run with the in-loop finite check: the checks only read the state
    m = c["long_n"]
    chk = run_gpu(gpu, w, phi0, pi0, m, tile=(c["rows"], c["wpb"]), steps_per_pass=2,
                  check_every=c["check_every"])
    ref = run_gpu(gpu, w, phi0, pi0, m, tile=(c["rows"], c["wpb"]), steps_per_pass=2)
    for k in range(3):
        if ref[k] is not None:
            assert np.array_equal(chk[k], ref[k]), (c, k)


@pytest.mark.parametrize("case", range(16))
def test_random_adjoint(gpu, case):
    c = _draw(7000 + case, 8, 1)
    nr, nth, n = c["nr"], c["nth"], c["n"]
    w = small_case(c["a"], c["s"], c["m"], nr, nth, ext=c["ext"])
    phi0, pi0 = inputs.random_state(nr, nth, seed=8000 + case)
    lam0 = inputs.random_state(nr, nth, seed=9000 + case)
    o = oracle.OracleGrid(c["a"], c["s"], c["m"], nr, nth, w["rstar_min"], w["rstar_max"], w["dt"])
    p, q = o.project(phi0, pi0)
    states = []
    for _ in range(n):
        states.append((p.copy(), q.copy()))
        p, q = o.step(p, q, 1)
    ref_p, ref_q, ref_dlda = oracle_segment_adjoint(o, states, lam0[0], lam0[1], c["gser"], w["extract_rstar"],
                                                    w["extract_theta"])
    g = gpu.TeukGrid(c["a"], c["s"], c["m"], nr, nth, w["rstar_min"], w["rstar_max"], w["dt"],
                     extract_rstar=w["extract_rstar"], extract_theta=w["extract_theta"])
    g.set_adjoint_tile(c["rows"], c["wpb"])
    g.set_initial_data(torch.from_numpy(phi0).cuda(), torch.from_numpy(pi0).cuda())
    win = g.new_window(n)
    g.step_store(n, win)
    gs = torch.from_numpy(c["gser"]).cuda()
    outs = []
    for spin, spp in ((True, 2), (False, 1), (False, 2)):
        g.set_steps_per_pass(spp)
        lp = torch.from_numpy(lam0[0].copy()).cuda()
        lq = torch.from_numpy(lam0[1].copy()).cuda()
        d = g.adjoint(n, lp, lq, gs, win if spin else None, spin=spin)
        torch.cuda.synchronize()
        outs.append((lp.cpu().numpy(), lq.cpu().numpy(), d))
    # the stored-tangent route over the same steps
    g.set_initial_data(torch.from_numpy(phi0).cuda(), torch.from_numpy(pi0).cuda())
    g.set_steps_per_pass(2)
    g.step_tangent(n, win)
    lp = torch.from_numpy(lam0[0].copy()).cuda()
    lq = torch.from_numpy(lam0[1].copy()).cuda()
    d = g.adjoint(n, lp, lq, gs, win, tangent=True)
    torch.cuda.synchronize()
    outs.append((lp.cpu().numpy(), lq.cpu().numpy(), d))
    g.close()
    for k in (1, 2, 3):
        assert np.array_equal(outs[0][0], outs[k][0]) and np.array_equal(outs[0][1], outs[k][1]), (c, k)
    assert rel_err(outs[0][0], ref_p) <= TOL and rel_err(outs[0][1], ref_q) <= TOL, c
    assert abs(outs[0][2] - ref_dlda) <= 1e-10 * abs(ref_dlda), (c, outs[0][2], ref_dlda)
    assert abs(outs[3][2] - ref_dlda) <= 1e-10 * abs(ref_dlda), (c, outs[3][2], ref_dlda)


@pytest.mark.parametrize("case", range(12))
def test_random_spin_tangent(gpu, case):
    c = _draw(11000 + case, 10, 0)
    nr, nth, n = c["nr"], c["nth"], c["n"]
    w = small_case(c["a"], c["s"], c["m"], nr, nth, ext=c["ext"])
    u0 = inputs.random_state(nr, nth, seed=12000 + case)
    v0 = inputs.random_state(nr, nth, seed=13000 + case)
    g = gpu.TeukGrid(w["a"], w["s"], w["m"], nr, nth, w["rstar_min"], w["rstar_max"], w["dt"],
                     extract_rstar=w["extract_rstar"], extract_theta=w["extract_theta"])
    g.set_adjoint_tile(c["rows"], c["wpb"])
    g.set_initial_data(torch.from_numpy(u0[0]).cuda(), torch.from_numpy(u0[1]).cuda())
    g.set_spin_tangent(torch.from_numpy(v0[0]).cuda(), torch.from_numpy(v0[1]).cuda())
    su, sv = g.step_spin_tangent(n)
    got = [x.cpu().numpy() for x in (*g.state(), *g.spin_tangent())]
    g.close()
    o = oracle.OracleGrid(c["a"], c["s"], c["m"], nr, nth, w["rstar_min"], w["rstar_max"], w["dt"])
    p, q = o.project(*u0)
    vp, vq = o.project(*v0)
    ref = o.evolve_spin_tangent(p, q, vp, vq, n, w["extract_rstar"], w["extract_theta"])
    for k in range(4):
        assert rel_err(got[k], ref[k]) <= TOL, (c, k)
    if c["ext"]:
        assert rel_err(su.cpu().numpy(), ref[4]) <= TOL and rel_err(sv.cpu().numpy(), ref[5]) <= TOL, c
    fwd = run_gpu(gpu, w, u0[0], u0[1], n, steps_per_pass=1)
    assert np.array_equal(fwd[0], got[0]) and np.array_equal(fwd[1], got[1]), c
    if c["ext"]:
        assert np.array_equal(fwd[2], su.cpu().numpy()), c


@pytest.mark.parametrize("case", range(8))
def test_random_batch(gpu, case):
    """2-6 members of random size and physics, a random launch shape and
    steps per pass, an odd or even step count: every member equals its
    single-grid evolution bit for bit, and the batch's samples equal the
    single grids' extraction."""
    rng = np.random.default_rng(11000 + case)
    members, data, ext = [], [], []
    for k in range(int(rng.integers(2, 7))):
        nr, nth = int(rng.integers(3, 500)), int(rng.integers(2, 70))
        a, s, m = float(rng.uniform(0, 0.99)), int(rng.choice([-2, 0, 2])), int(rng.integers(-4, 5))
        r0 = float(rng.uniform(-60.0, 0.0))
        r1 = r0 + float(rng.uniform(20.0, 120.0))
        dt = inputs.stable_dt((r1 - r0) / (nr - 1), nth, m, s, 50)
        pts = [(float(rng.uniform(r0, r1)), float(rng.uniform(0, math.pi))) for _ in range(int(rng.integers(0, 3)))]
        members.append(dict(a=a, s=s, m=m, nr=nr, ntheta=nth, rstar_min=r0, rstar_max=r1, dt=dt,
                            extract_rstar=[p[0] for p in pts], extract_theta=[p[1] for p in pts]))
        data.append(inputs.random_state(nr, nth, seed=12000 + 10 * case + k))
        ext.append(pts)
    rows, wpb = int(rng.integers(1, 80)), int(rng.choice([1, 2, 4]))
    blocks = int(rng.integers(1, 2049))
    spp, n = int(rng.choice([1, 2])), int(rng.integers(1, 9))
    b = gpu.TeukBatch(members)
    b.set_launch(rows, wpb, blocks)
    b.set_steps_per_pass(spp)
    for k, (p, q) in enumerate(data):
        b.set_initial_data(k, torch.from_numpy(p).cuda(), torch.from_numpy(q).cuda())
    b.step(n)
    got = [[t.cpu().numpy() for t in b.state(k)] for k in range(len(members))]
    samples = b.extract().cpu().numpy() if b.n_extract() else None
    b.close()
    off = 0
    for k, mb in enumerate(members):
        g = gpu.TeukGrid(mb["a"], mb["s"], mb["m"], mb["nr"], mb["ntheta"], mb["rstar_min"], mb["rstar_max"],
                         mb["dt"])
        g.set_initial_data(torch.from_numpy(data[k][0]).cuda(), torch.from_numpy(data[k][1]).cuda())
        g.step(n)
        ref = [t.cpu().numpy() for t in g.state()]
        if ext[k]:
            want = g.extract([p[0] for p in ext[k]], [p[1] for p in ext[k]]).cpu().numpy()
            assert np.array_equal(samples[off:off + len(ext[k])], want), (case, k)
            off += len(ext[k])
        g.close()
        assert np.array_equal(got[k][0], ref[0]) and np.array_equal(got[k][1], ref[1]), (case, k, rows, wpb, blocks)
