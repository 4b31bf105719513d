"""Differentiable evolution: extraction series as a function of the initial
data (Phi0, Pi0) and of the spin a, with checkpoint/recompute.

Forward: the state is copied to a checkpoint every K steps while the
library advances the grid (teuk_step_n).  Backward, for each segment from the
last to the first: restore its checkpoint, recompute its K steps while the
library keeps their input states in a window (teuk_step_n_store), and run the
library's adjoint over the segment (teuk_adjoint_step_n), which carries the
cotangent of the state and accumulates dL/da.  Device memory: the
checkpoints (one state per K steps) plus one window of K states.

When the spin needs no gradient, no checkpoints are kept and the backward
is one adjoint sweep over all steps: the cotangents of the linear step do
not depend on the forward states, so nothing is recomputed.

Gradients follow PyTorch's convention for complex tensors
(dL/dRe + i dL/dIm).  All arithmetic runs in the library's HIP kernels; this
module only moves tensors and handles between the calls.
"""
import torch

from . import binding


def _make_grid(a, cfg):
    return binding.TeukGrid(a, cfg["s"], cfg["m"], cfg["nr"], cfg["ntheta"], cfg["rstar_min"], cfg["rstar_max"],
                            cfg["dt"], extract_rstar=cfg.get("extract_rstar", ()),
                            extract_theta=cfg.get("extract_theta", ()))


class TeukEvolve(torch.autograd.Function):
    """series = TeukEvolve.apply(phi0, pi0, a, cfg, n_steps, checkpoint_every)

    phi0, pi0: complex128 (ntheta, nr) on the GPU; a: 0-dim float64 tensor;
    cfg: dict with s, m, nr, ntheta, rstar_min, rstar_max, dt, extract_rstar,
    extract_theta.  Returns the extraction series, complex128 (n_steps, n_extract)."""

    @staticmethod
    def forward(ctx, phi0, pi0, a, cfg, n_steps, checkpoint_every):
        n, K = int(n_steps), int(checkpoint_every)
        if n < 1 or K < 1:
            raise ValueError("need n_steps >= 1 and checkpoint_every >= 1")
        grid = _make_grid(float(a), cfg)
        if grid.n_extract < 1:
            raise ValueError("the loss is a function of the extraction series: give extraction points")
        grid.set_initial_data(phi0.detach(), pi0.detach())
        series = torch.empty((n, grid.n_extract), dtype=torch.complex128, device=grid.device)
        need_a = ctx.needs_input_grad[2]
        ckpts = []
        if need_a:
            for k in range(0, n, K):
                m = min(K, n - k)
                ckpts.append(grid.state())
                binding.teuk_step_n(grid.handle, m, series[k:k + m])
        else:
            binding.teuk_step_n(grid.handle, n, series)
        ctx.grid, ctx.ckpts, ctx.n, ctx.K, ctx.need_a = grid, ckpts, n, K, need_a
        ctx.a_meta = (a.dtype, a.device, a.shape)
        return series

    @staticmethod
    def backward(ctx, gseries):
        grid, n, K = ctx.grid, ctx.n, ctx.K
        grid.enable_adjoint()
        gseries = gseries.to(dtype=torch.complex128).contiguous()
        lam_phi = torch.zeros(grid.shape, dtype=torch.complex128, device=grid.device)
        lam_pi = torch.zeros_like(lam_phi)
        grad_a = None
        if ctx.need_a:
            window = grid.new_window(min(K, n))
            dlda = 0.0
            segs = [(k, min(K, n - k)) for k in range(0, n, K)]
            for idx in range(len(segs) - 1, -1, -1):
                k, m = segs[idx]
                grid.set_initial_data(*ctx.ckpts[idx])
                grid.step_store(m, window, series=False)
                dlda += grid.adjoint(m, lam_phi, lam_pi, gseries[k:k + m], window, project_initial=(idx == 0))
            dtype, device, shape = ctx.a_meta
            grad_a = torch.full(shape, dlda, dtype=dtype, device=device)
        else:
            grid.adjoint(n, lam_phi, lam_pi, gseries, None, project_initial=True, spin=False)
        ctx.grid = None
        ctx.ckpts = None
        grid.close()
        return lam_phi, lam_pi, grad_a, None, None, None


def evolve(phi0, pi0, a, cfg, n_steps, checkpoint_every=100):
    """Extraction series of an n-step evolution, differentiable in phi0, pi0 and a."""
    if not torch.is_tensor(a):
        a = torch.tensor(float(a), dtype=torch.float64, device=phi0.device)
    return TeukEvolve.apply(phi0, pi0, a, cfg, n_steps, checkpoint_every)
