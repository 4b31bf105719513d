"""Shared helpers of the GPU parity tests: run the same seeded input through
the HIP library (C ABI) and through the oracle, and compare."""
import math

import numpy as np

import oracle
from paper_1010_3816_amd import inputs


def rel_err(gpu, ref):
    """Normwise relative error: max |gpu - ref| / max |ref| over all entries."""
    ref = np.asarray(ref)
    scale = np.max(np.abs(ref))
    return float(np.max(np.abs(np.asarray(gpu) - ref)) / (scale if scale > 0 else 1.0))


def run_gpu(binding, w, phi0, pi0, n, tile=None, coef=None, mode=None, steps_per_pass=None, check_every=None,
            cache_policy=None, block_steps=None, block_cols=0):
    import torch

    g = binding.TeukGrid(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["dt"],
                         coef_mode=binding.TEUK_COEF_USER if coef is not None else binding.TEUK_COEF_KERR,
                         extract_rstar=w.get("extract_rstar", []), extract_theta=w.get("extract_theta", []))
    if coef is not None:
        g.set_coefficients(torch.from_numpy(coef[0]).cuda(), torch.from_numpy(coef[1]).cuda())
    if tile is not None:
        g.set_tile(*tile)
    if steps_per_pass is not None:
        g.set_steps_per_pass(steps_per_pass)
    if check_every is not None:
        g.set_finite_check(check_every)
    if cache_policy is not None:
        g.set_cache_policy(cache_policy)
    # A test that picks the sweeps' launch shape or steps per pass is about
    # the sweeps: the small-grid block pass is off unless asked for.
    if block_steps is None and (steps_per_pass is not None or tile is not None):
        block_steps = 0
    if block_steps is not None:
        g.set_block_launch(block_steps, block_cols)
    g.set_initial_data(torch.from_numpy(phi0).cuda(), torch.from_numpy(pi0).cuda())
    ser = g.step(n)
    phi, pi = g.state()
    torch.cuda.synchronize()
    out = (phi.cpu().numpy(), pi.cpu().numpy(), None if ser is None else ser.cpu().numpy())
    g.close()
    return out


def run_oracle(w, phi0, pi0, n, coef=None):
    o = oracle.OracleGrid(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["dt"],
                          kerr=coef is None)
    if coef is not None:
        o.set_coefficients(*coef)
    p, q = o.project(phi0, pi0)
    p, q, ser = o.evolve(p, q, n, w.get("extract_rstar", []), w.get("extract_theta", []))
    return p, q, ser


def small_case(a, s, m, nr, nth, rmin=-30.0, rmax=60.0, dt=None, ext=((20.0, math.pi / 2),)):
    dr = (rmax - rmin) / (nr - 1)
    w = dict(a=a, s=s, m=m, nr=nr, ntheta=nth, rstar_min=rmin, rstar_max=rmax,
             extract_rstar=[e[0] for e in ext], extract_theta=[e[1] for e in ext])
    w["dt"] = dt if dt is not None else inputs.stable_dt(dr, nth, m, s, 200)
    return w


def oracle_segment_adjoint(o, states, lam_phi, lam_pi, gser, ext_r, ext_t):
    """Reverse of one segment with oracle primitives: `states` are the inputs
    of the segment's steps; gser[k] is dL/d(sample after step k+1)."""
    n = len(states)
    lp, lq = np.array(lam_phi, dtype=np.complex128), np.array(lam_pi, dtype=np.complex128)
    if gser is not None:
        for e in range(len(ext_r)):
            lp = o.extract_adjoint(lp, ext_r[e], ext_t[e], gser[n - 1, e])
    dlda = 0.0
    for k in range(n - 1, -1, -1):
        tp, tq = o.tangent_a(*states[k])
        dlda += float(np.real(np.vdot(lp, tp) + np.vdot(lq, tq)))
        lp, lq = o.adjoint_step(lp, lq)
        if gser is not None and k >= 1:
            for e in range(len(ext_r)):
                lp = o.extract_adjoint(lp, ext_r[e], ext_t[e], gser[k - 1, e])
    return lp, lq, dlda
