"""Batched evolutions (C ABI teuk_batch_*): every member must equal, bit for
bit, a single-grid evolution of the same problem (the per-point arithmetic
does not depend on the launch), and hence the oracle within the forward
tolerance; step parity, graph replay and relaunch shapes must not change
results."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1010_3816_amd import autotune, inputs
from parity import rel_err

pytestmark = pytest.mark.gpu


def _members():
    base = [
        (0.0, -2, 2, 130, 20, -30.0, 60.0),
        (0.7, -2, 1, 201, 17, -40.0, 80.0),
        (0.9, 0, -3, 187, 70, -20.0, 50.0),
        (0.99, -1, 4, 64, 9, -10.0, 30.0),
        (0.3, 0, 0, 3, 2, 0.0, 1.0),
        (0.5, -2, 2, 500, 33, -50.0, 150.0),
    ]
    out = []
    for a, s, m, nr, nth, r0, r1 in base:
        dr = (r1 - r0) / (nr - 1)
        out.append(dict(a=a, s=s, m=m, nr=nr, ntheta=nth, rstar_min=r0, rstar_max=r1,
                        dt=inputs.stable_dt(dr, nth, m, s, 200)))
    return out


def _single(gpu, mb, phi0, pi0, n):
    g = gpu.TeukGrid(mb["a"], mb["s"], mb["m"], mb["nr"], mb["ntheta"], mb["rstar_min"], mb["rstar_max"], mb["dt"])
    g.set_initial_data(torch.from_numpy(phi0).cuda(), torch.from_numpy(pi0).cuda())
    g.step(n)
    out = [t.cpu().numpy() for t in g.state()]
    g.close()
    return out


def test_members_equal_single_grids(gpu):
    mbs = _members()
    data = [inputs.random_state(m["nr"], m["ntheta"], seed=100 + k) for k, m in enumerate(mbs)]
    b = gpu.TeukBatch(mbs)
    for k, (p, q) in enumerate(data):
        b.set_initial_data(k, torch.from_numpy(p).cuda(), torch.from_numpy(q).cuda())
    for n in (1, 4, 2, 3):       # odd and even runs: parity changes and graph replays
        b.step(n)
    got = [[t.cpu().numpy() for t in b.state(k)] for k in range(len(mbs))]
    for k, mb in enumerate(mbs):
        ref = _single(gpu, mb, data[k][0], data[k][1], 10)
        assert np.array_equal(got[k][0], ref[0]) and np.array_equal(got[k][1], ref[1]), k
    # one member against the oracle
    mb = mbs[1]
    o = oracle.OracleGrid(mb["a"], mb["s"], mb["m"], mb["nr"], mb["ntheta"], mb["rstar_min"], mb["rstar_max"], mb["dt"])
    p, q = o.project(*data[1])
    p, q = o.step(p, q, 10)
    assert rel_err(got[1][0], p) <= 1e-11 and rel_err(got[1][1], q) <= 1e-11
    b.close()


@pytest.mark.parametrize("launch", [(1, 1, 7), (3, 2, 64), (16, 8, 512), (64, 4, 2048), (128, 1, 4096)])
def test_launch_shapes_identical(gpu, launch):
    mbs = _members()
    data = [inputs.random_state(m["nr"], m["ntheta"], seed=200 + k) for k, m in enumerate(mbs)]
    res = []
    for shape in [None, launch]:
        b = gpu.TeukBatch(mbs)
        if shape is not None:
            b.set_launch(*shape)
        for k, (p, q) in enumerate(data):
            b.set_initial_data(k, torch.from_numpy(p).cuda(), torch.from_numpy(q).cuda())
        b.step(5)
        res.append([[t.cpu().numpy() for t in b.state(k)] for k in range(len(mbs))])
        b.close()
    for k in range(len(mbs)):
        assert np.array_equal(res[0][k][0], res[1][k][0]) and np.array_equal(res[0][k][1], res[1][k][1])


def test_batch64_workload_sampled_members(gpu):
    """The 64-member workload: a few steps of the whole batch, three members
    checked against single-grid runs."""
    mbs = inputs.batch_members()
    b = gpu.TeukBatch(mbs)
    for k, mb in enumerate(mbs):
        p, q = inputs.initial_data(mb)
        b.set_initial_data(k, torch.from_numpy(p).cuda(), torch.from_numpy(q).cuda())
    b.step(3)
    assert b.total_points() == sum(m["nr"] * m["ntheta"] for m in mbs)
    for k in (0, 31, 63):
        p, q = inputs.initial_data(mbs[k])
        ref = _single(gpu, mbs[k], p, q, 3)
        got = [t.cpu().numpy() for t in b.state(k)]
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    b.close()


def test_autotuners_pick_valid_shapes(gpu, tmp_path, monkeypatch):
    monkeypatch.setenv("TEUK_TUNE_CACHE", str(tmp_path / "launch.json"))
    w = inputs.workload("kerr_a0.9_6400x256")
    g = gpu.TeukGrid(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["dt"])
    res = autotune.tune_grid(g, rows=(8, 16), waves=(2, 4), steps=5)
    assert g.tile() == (res["rows"], res["waves"])
    again = autotune.tune_grid(g, rows=(8, 16), waves=(2, 4), steps=5)
    assert again.get("cached") and (again["rows"], again["waves"]) == (res["rows"], res["waves"])
    assert res["block"] == 0 and g.block_steps() == 0  # 256 rows: no block pass
    g.close()
    # a small grid: sweeps' shapes with the block pass off, and its steps per launch
    g = gpu.TeukGrid(0.0, -2, 2, 400, 32, -50.0, 150.0, 0.01)
    res = autotune.tune_grid(g, rows=(1, 4), waves=(1,), steps=5)
    kinds = {e["block"] for e in res["table"]}
    assert 0 in kinds and len(kinds) > 1, kinds
    assert g.tile() == (res["rows"], res["waves"]) and g.block_steps() == res["block"]
    cands = autotune.block_candidates(400, 32, torch.cuda.get_device_properties(0).multi_processor_count)
    assert res["block"] == 0 or (res["block"], res["cols"]) in cands
    if res["block"]:
        assert g.block_launch() == (res["block"], res["cols"])
    again = autotune.tune_grid(g, rows=(1, 4), waves=(1,), steps=5)
    assert again.get("cached") and again["block"] == res["block"] and g.block_steps() == res["block"]
    g.close()
    b = gpu.TeukBatch(_members())
    res = autotune.tune_batch(b, rows=(8, 16), waves=(4,), blocks_per_cu=(1, 2), steps=3)
    assert b.launch() == (res["rows"], res["waves"], res["blocks"])
    b.close()


def test_two_step_launches_identical(gpu):
    """Two steps per launch (the default) against one step per launch, over
    runs of odd and even lengths (parity changes, graph replays, a single
    last step), bit for bit."""
    mbs = _members()
    data = [inputs.random_state(m["nr"], m["ntheta"], seed=300 + k) for k, m in enumerate(mbs)]
    res = []
    for spp in (1, 2):
        b = gpu.TeukBatch(mbs)
        b.set_steps_per_pass(spp)
        for k, (p, q) in enumerate(data):
            b.set_initial_data(k, torch.from_numpy(p).cuda(), torch.from_numpy(q).cuda())
        for n in (1, 5, 2, 3, 4):
            b.step(n)
        res.append([[t.cpu().numpy() for t in b.state(k)] for k in range(len(mbs))])
        b.close()
    for k in range(len(mbs)):
        assert np.array_equal(res[0][k][0], res[1][k][0]) and np.array_equal(res[0][k][1], res[1][k][1]), k


def test_batch64_full_length(gpu):
    """The 64-member workload for all its 5000 steps in the default launch:
    every member equals its single-grid evolution bit for bit, and the last
    step of three members equals one oracle step taken from the batch's state
    before it."""
    mbs = inputs.batch_members()
    n = mbs[0]["steps"]
    b = gpu.TeukBatch(mbs)
    for k, mb in enumerate(mbs):
        p, q = inputs.initial_data(mb)
        b.set_initial_data(k, torch.from_numpy(p).cuda(), torch.from_numpy(q).cuda())
    b.step(n - 1)
    sampled = (0, 37, 63)
    before = {k: [t.cpu().numpy() for t in b.state(k)] for k in sampled}
    b.step(1)
    for k, mb in enumerate(mbs):
        g = gpu.TeukGrid(mb["a"], mb["s"], mb["m"], mb["nr"], mb["ntheta"], mb["rstar_min"], mb["rstar_max"],
                         mb["dt"])
        p, q = inputs.initial_data(mb)
        g.set_initial_data(torch.from_numpy(p).cuda(), torch.from_numpy(q).cuda())
        g.step(n)
        ref, got = g.state(), b.state(k)
        assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1]), k
        g.close()
        if k in sampled:
            o = oracle.OracleGrid(mb["a"], mb["s"], mb["m"], mb["nr"], mb["ntheta"], mb["rstar_min"],
                                  mb["rstar_max"], mb["dt"])
            op, oq = o.step(before[k][0], before[k][1], 1)
            after = [t.cpu().numpy() for t in got]
            assert np.isfinite(after[0]).all() and np.isfinite(after[1]).all()
            assert rel_err(after[0], op) <= 1e-11 and rel_err(after[1], oq) <= 1e-11, k
    b.close()
