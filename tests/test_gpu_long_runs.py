"""Full-length parity of the forward evolution against the oracle, on the
standard full-size grids, from their own initial data, in the default launch
configuration (two Lax-Wendroff steps per pass, default tiles).

 * Kerr a = 0.9, 6400 x 256: all 20,000 steps on the whole grid.  The oracle
   runs beside it chunk by chunk (one to three minutes on the host threads);
   the states are compared after every chunk, the whole extraction series at
   the end.  Besides the workload's own extraction point (r* = 500, which no
   signal reaches in t = 23.2 at the stable time step) the run samples points
   the pulse does reach.  This run amplifies rounding: a second GPU copy
   started from data perturbed by one ulp drifts from the first by d_k
   (measured here in lockstep; 3e-13 after 2000 steps, 7e-12 after 20,000),
   and any two correctly rounded FP64 implementations drift apart by a small
   multiple of it.  The bar at chunk k is therefore max(1e-11, 4 d_k): the
   1e-11 of the forward step wherever the run's own rounding floor is below
   it, four times that floor where it is not.
 * Kerr a = 0.99, 25600 x 512: 1000 steps of the full grid, compared with
   the oracle on windows of 3000 columns (the pulse, both radial ends of a
   random state and its middle) where the windows' own edges, zeroed like
   radial boundaries, cannot have reached (one column per step).

Bar: normwise relative error <= 1e-11 (the parity bound of the forward step),
with the derived floor above for the 20,000-step run.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1010_3816_amd import inputs
from parity import rel_err

TOL = 1e-11
pytestmark = pytest.mark.gpu


@pytest.mark.timeout(1200)
def test_kerr_6400x256_all_steps_against_oracle(gpu, progress):
    import torch

    w = dict(inputs.workload("kerr_a0.9_6400x256"))
    n, chunk = w["steps"], 2000
    t_end = n * w["dt"]
    # the workload's point, then two the pulse reaches (centre + t/2, on and off the equator)
    ext_r = w["extract_rstar"] + [w["center"] + 0.5 * t_end, w["center"] + 0.3 * t_end]
    ext_t = w["extract_theta"] + [math.pi / 2, 1.1]
    phi0, pi0 = inputs.initial_data(w)
    # one-ulp perturbation of the initial data (random signs, seeded)
    rng = np.random.default_rng(7)

    def ulp(x):
        return x + (np.spacing(np.abs(x.real)) * rng.choice([-1.0, 1.0], x.shape)
                    + 1j * np.spacing(np.abs(x.imag)) * rng.choice([-1.0, 1.0], x.shape))

    grids = []
    for p0, q0 in ((phi0, pi0), (ulp(phi0), ulp(pi0))):
        g = gpu.TeukGrid(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["dt"],
                         extract_rstar=ext_r, extract_theta=ext_t)
        assert g.steps_per_pass() == 2
        g.set_initial_data(torch.from_numpy(p0).cuda(), torch.from_numpy(q0).cuda())
        grids.append(g)
    g, gpert = grids
    o = oracle.OracleGrid(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["dt"])
    p, q = o.project(phi0, pi0)
    gser, oser = [], []
    worst, bar = 0.0, TOL
    for k0 in range(0, n, chunk):
        gser.append(g.step(chunk).cpu().numpy())
        gpert.step(chunk, series=False)
        gp, gq = (t.cpu().numpy() for t in g.state())
        pp, pq = (t.cpu().numpy() for t in gpert.state())
        d = max(rel_err(pp, gp), rel_err(pq, gq))  # the run's own rounding floor
        p, q, s = o.evolve(p, q, chunk, ext_r, ext_t)
        oser.append(s)
        e = max(rel_err(gp, p), rel_err(gq, q))
        bar = max(TOL, 4.0 * d)
        worst = max(worst, e)
        progress(f"[long-run] 6400x256 steps {k0 + chunk}/{n}: state rel err {e:.2e}, "
             f"one-ulp drift {d:.2e}, bar {bar:.2e}")
        assert e <= bar, (k0 + chunk, e, d)
    gpert.close()
    gser, oser = np.concatenate(gser), np.concatenate(oser)
    assert gser.shape == (n, 3)
    assert rel_err(gser, oser) <= bar
    # the points the pulse reaches carry the signal the comparison is about
    assert np.max(np.abs(oser[:, 1])) > 1e-3 * np.max(np.abs(phi0))
    assert np.max(np.abs(oser[:, 2])) > 1e-3 * np.max(np.abs(phi0))
    progress(f"[long-run] 6400x256 worst state rel err {worst:.2e}, series {rel_err(gser, oser):.2e} (bar {bar:.2e})")
    g.close()


def _window_check(w, phi0, pi0, got, n, i0, width, progress):
    """The oracle on columns i0 .. i0+width-1 of the grid for n steps against
    the GPU's state there, where the window's artificial edges cannot reach."""
    nr = w["nr"]
    i1 = i0 + width - 1
    dr = (w["rstar_max"] - w["rstar_min"]) / (nr - 1)
    o = oracle.OracleGrid(w["a"], w["s"], w["m"], width, w["ntheta"], w["rstar_min"] + i0 * dr,
                          w["rstar_min"] + i1 * dr, w["dt"])
    p, q = o.project(phi0[:, i0:i1 + 1], pi0[:, i0:i1 + 1])
    p, q = o.step(p, q, n)
    lo = 0 if i0 == 0 else n + 1
    hi = width if i1 == nr - 1 else width - n - 1
    e = max(rel_err(got[0][:, i0:i1 + 1][:, lo:hi], p[:, lo:hi]),
            rel_err(got[1][:, i0:i1 + 1][:, lo:hi], q[:, lo:hi]))
    progress(f"[long-run] 25600x512 window {i0}..{i1} (columns {lo}..{hi - 1} compared): rel err {e:.2e}")
    assert e <= TOL, (i0, e)


@pytest.mark.timeout(900)
def test_kerr_25600x512_windows_against_oracle(gpu, progress):
    import torch

    w = inputs.workload("kerr_a0.99_25600x512")
    n, width = 1000, 3000
    nr, nth = w["nr"], w["ntheta"]
    dr = (w["rstar_max"] - w["rstar_min"]) / (nr - 1)
    pulse, rnd = inputs.initial_data(w), inputs.random_state(nr, nth, seed=1011)
    for name, (phi0, pi0), starts in (("pulse", pulse, [int((w["center"] - w["rstar_min"]) / dr) - width // 2]),
                                      ("random", rnd, [0, nr // 2 - width // 2, nr - width])):
        g = gpu.TeukGrid(w["a"], w["s"], w["m"], nr, nth, w["rstar_min"], w["rstar_max"], w["dt"])
        g.set_initial_data(torch.from_numpy(phi0).cuda(), torch.from_numpy(pi0).cuda())
        g.step(n)
        got = [t.cpu().numpy() for t in g.state()]
        g.close()
        assert np.isfinite(got[0]).all() and np.isfinite(got[1]).all()
        progress(f"[long-run] 25600x512 {name} data: {n} steps on the GPU done")
        for i0 in starts:
            _window_check(w, phi0, pi0, got, n, i0, width, progress)
