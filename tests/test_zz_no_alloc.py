"""The allocation-free extraction entry point (teuk_extract_noalloc) against
teuk_extract through the C ABI: same points, same state, bit-identical
samples, on two calls in a row (the second with fewer points), and the
oracle's bilinear samples of the same state within the parity bound."""
import math

import numpy as np
import pytest

from paper_1010_3816_amd import inputs
from parity import rel_err, small_case

import oracle

TOL = 1e-11


def _points(rng, n, rmin, rmax):
    r = rng.uniform(rmin, rmax, n)
    t = rng.uniform(0.0, math.pi, n)
    # grid ends and poles, where the ghost rows enter the weights
    fixed_r = [rmin, rmax, rmin, rmax, 0.5 * (rmin + rmax)]
    fixed_t = [0.0, math.pi, math.pi, 0.0, 0.01]
    k = min(n, len(fixed_r))
    r[:k], t[:k] = fixed_r[:k], fixed_t[:k]
    return r, t


@pytest.mark.gpu
def test_extract_noalloc_matches_extract(gpu):
    import torch

    w = small_case(0.7, -2, 3, 210, 27, ext=())
    phi0, pi0 = inputs.random_state(210, 27, seed=77)
    g = gpu.TeukGrid(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["dt"])
    g.set_initial_data(torch.from_numpy(phi0).cuda(), torch.from_numpy(pi0).cuda())
    g.step(7)
    phi, pi = g.state()
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    o = oracle.OracleGrid(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["dt"])
    state = phi.cpu().numpy()
    for n in (300, 7):  # more points than one staging chunk, then fewer
        r, t = _points(rng, n, w["rstar_min"], w["rstar_max"])
        ref = torch.empty(n, dtype=torch.complex128, device="cuda")
        got = torch.full((n,), complex(float("nan"), float("nan")), dtype=torch.complex128, device="cuda")
        gpu.teuk_extract(g.handle, r, t, ref)
        gpu.teuk_extract_noalloc(g.handle, r, t, got)
        torch.cuda.synchronize()
        a, b = ref.cpu().numpy(), got.cpu().numpy()
        assert np.array_equal(a, b), (n, np.max(np.abs(a - b)))
        want = np.array([o.extract(state, r[e], t[e]) for e in range(n)])
        assert rel_err(b, want) <= TOL
    # the size limit is checked on the host, before any device work
    with pytest.raises(gpu.TeukError) as ei:
        gpu.teuk_extract_noalloc(g.handle, np.zeros(4097), np.zeros(4097),
                                 torch.empty(4097, dtype=torch.complex128, device="cuda"))
    assert ei.value.code == gpu.TEUK_E_INVALID_ARG
    g.close()
