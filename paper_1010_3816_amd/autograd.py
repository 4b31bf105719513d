"""Differentiable evolution: extraction series as a function of the initial
data (Phi0, Pi0) and of the spin a.

The spin is one scalar, so its derivative can also run forward: with
spin="forward" (the default) the library advances v = du/da beside the
state by the tangent-linear step (teuk_step_n_spin_tangent) and keeps the
samples of v, ds/da; the backward forms dL/da = sum Re <dL/ds, ds/da>
(teuk_spin_gradient), and the initial-data gradients come from one adjoint
sweep over all steps without forward states.  No checkpoints, no recompute.

With spin="reverse", checkpoint/recompute.  Forward: the state is copied
to a checkpoint every K steps while the library advances the grid
(teuk_step_n).  Backward, for each segment from the
last to the first: restore its checkpoint, recompute its K steps while the
library keeps, for each step k, its derivative with respect to the spin at
fixed input, T_k = (dA/da) u^k, in a window (teuk_step_n_tangent), and run the
library's adjoint over the segment (teuk_adjoint_step_n), which carries the
cotangent of the state and accumulates dL/da = sum_k Re <lambda^{k+1}, T_k>
from the cotangents it computes anyway.  Device memory: the checkpoints (one
state per K steps) plus one window of K states.  tangent=False keeps the
input states in the window instead (teuk_step_n_store) and lets the adjoint
recompute the spin term from them: the same gradient, by another route.

With overlap (the default) the recompute of the next segment runs on a
second grid and stream while the adjoint of the current one runs, into the
other of two windows: the two passes share the device better than they run
one after the other.  dL/da accumulates on the device (one partial sum per
segment, added in segment order) and the window handed back and forth is
guarded by events, so the host never waits inside the reverse pass and the
device is never left idle while it enqueues the next segment.  The
arithmetic and the order of the dL/da sums are unchanged, so the gradients
are the same bit for bit.  Device memory: one more window.

When the spin needs no gradient, no checkpoints are kept and the backward
is one adjoint sweep over all steps: the cotangents of the linear step do
not depend on the forward states, so nothing is recomputed.

Gradients follow PyTorch's convention for complex tensors
(dL/dRe + i dL/dIm).  All arithmetic runs in the library's HIP kernels; this
module only moves tensors and handles between the calls.
"""
import torch

from . import binding


def _make_grid(a, cfg, stream=None):
    return binding.TeukGrid(a, cfg["s"], cfg["m"], cfg["nr"], cfg["ntheta"], cfg["rstar_min"], cfg["rstar_max"],
                            cfg["dt"], extract_rstar=cfg.get("extract_rstar", ()),
                            extract_theta=cfg.get("extract_theta", ()), stream=stream)


def _recompute(grid, m, window, tangent):
    if tangent:
        grid.step_tangent(m, window)
    else:
        grid.step_store(m, window, series=False)


def _reverse_sequential(grid, ckpts, segs, K, gseries, lam_phi, lam_pi, tangent):
    window = grid.new_window(K)
    dlda = grid.torch.zeros((), dtype=grid.torch.float64, device=grid.device)
    for idx in range(len(segs) - 1, -1, -1):
        k, m = segs[idx]
        grid.set_initial_data(*ckpts[idx])
        _recompute(grid, m, window, tangent)
        grid.adjoint(m, lam_phi, lam_pi, gseries[k:k + m], window, project_initial=(idx == 0), tangent=tangent,
                     accum=dlda)
    return dlda


def _reverse_overlapped(grid, a, cfg, ckpts, segs, K, gseries, lam_phi, lam_pi, tangent):
    """Segments in reverse; the recompute of segment idx-1 (second grid, own
    stream, window (idx-1) % 2) is queued before the adjoint of segment idx
    (this grid's stream, window idx % 2), which waits (an event) for its own
    recompute only.  A recompute rewrites a window two segments after it was
    filled, and waits (an event) for the adjoint that read it.  Nothing here
    waits on the host."""
    torch = grid.torch
    rs = torch.cuda.Stream(device=grid.device)  # default priority
    rs.wait_stream(grid.stream)                 # the checkpoints were written on the forward stream
    rec = _make_grid(a, cfg, stream=rs)
    windows = [grid.new_window(K), grid.new_window(K)]
    done = [torch.cuda.Event(), torch.cuda.Event()]       # window filled
    released = [torch.cuda.Event(), torch.cuda.Event()]   # window read by its adjoint

    def recompute(idx, after_adjoint):
        m = segs[idx][1]
        if after_adjoint:
            rs.wait_event(released[idx % 2])
        rec.set_initial_data(*ckpts[idx])
        _recompute(rec, m, windows[idx % 2], tangent)
        done[idx % 2].record(rs)

    dlda = torch.zeros((), dtype=torch.float64, device=grid.device)
    last = len(segs) - 1
    recompute(last, False)
    for idx in range(last, -1, -1):
        if idx > 0:
            recompute(idx - 1, idx + 1 <= last)  # its window was last read by the adjoint of segment idx+1
        grid.stream.wait_event(done[idx % 2])
        k, m = segs[idx]
        grid.adjoint(m, lam_phi, lam_pi, gseries[k:k + m], windows[idx % 2], project_initial=(idx == 0),
                     tangent=tangent, accum=dlda)
        released[idx % 2].record(grid.stream)
    grid.stream.wait_stream(rs)  # the second grid's work is done before it is released
    torch.cuda.current_stream(grid.device).wait_stream(grid.stream)
    rec.close()
    return dlda


class TeukEvolve(torch.autograd.Function):
    """series = TeukEvolve.apply(phi0, pi0, a, cfg, n_steps, checkpoint_every, overlap, tangent, spin)

    phi0, pi0: complex128 (ntheta, nr) on the GPU; a: 0-dim float64 tensor;
    cfg: dict with s, m, nr, ntheta, rstar_min, rstar_max, dt, extract_rstar,
    extract_theta.  Returns the extraction series, complex128 (n_steps, n_extract).
    overlap: run the recompute of the next segment beside the adjoint of the
    current one (same results).  tangent: the recompute stores the step
    tangents (default) or the states (the same gradient, by another route).
    spin: "forward" (the spin derivative carried forward; checkpoint_every,
    overlap and tangent unused) or "reverse" (checkpointed adjoint)."""

    @staticmethod
    def forward(ctx, phi0, pi0, a, cfg, n_steps, checkpoint_every, overlap=True, tangent=True, spin="forward"):
        n, K = int(n_steps), int(checkpoint_every)
        if n < 1 or K < 1:
            raise ValueError("need n_steps >= 1 and checkpoint_every >= 1")
        if spin not in ("forward", "reverse"):
            raise ValueError("spin must be 'forward' or 'reverse'")
        grid = _make_grid(float(a), cfg)
        if grid.n_extract < 1:
            raise ValueError("the loss is a function of the extraction series: give extraction points")
        grid.set_initial_data(phi0.detach(), pi0.detach())
        series = torch.empty((n, grid.n_extract), dtype=torch.complex128, device=grid.device)
        need_a = ctx.needs_input_grad[2]
        ckpts = []
        ctx.tseries = None
        if need_a and spin == "forward":
            grid.set_spin_tangent()  # v = du/da = 0: the initial data do not depend on a
            ctx.tseries = torch.empty_like(series)
            binding.teuk_step_n_spin_tangent(grid.handle, n, series, ctx.tseries)
        elif need_a:
            for k in range(0, n, K):
                m = min(K, n - k)
                ckpts.append(grid.state())
                binding.teuk_step_n(grid.handle, m, series[k:k + m])
        else:
            binding.teuk_step_n(grid.handle, n, series)
        ctx.grid, ctx.ckpts, ctx.n, ctx.K, ctx.need_a = grid, ckpts, n, K, need_a
        ctx.cfg, ctx.overlap, ctx.a_val, ctx.tangent = cfg, bool(overlap), float(a), bool(tangent)
        ctx.spin = spin
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
        dtype, device, shape = ctx.a_meta
        if ctx.need_a and ctx.spin == "forward":
            dlda = torch.zeros((), dtype=torch.float64, device=grid.device)
            binding.teuk_spin_gradient(grid.handle, n, gseries, ctx.tseries, dlda)
            grad_a = dlda.to(dtype=dtype, device=device).reshape(shape)
            if ctx.needs_input_grad[0] or ctx.needs_input_grad[1]:
                grid.adjoint(n, lam_phi, lam_pi, gseries, None, project_initial=True, spin=False)
            ctx.tseries = None
        elif ctx.need_a:
            segs = [(k, min(K, n - k)) for k in range(0, n, K)]
            if ctx.overlap and len(segs) > 1:
                dlda = _reverse_overlapped(grid, ctx.a_val, ctx.cfg, ctx.ckpts, segs, min(K, n), gseries, lam_phi,
                                           lam_pi, ctx.tangent)
            else:
                dlda = _reverse_sequential(grid, ctx.ckpts, segs, min(K, n), gseries, lam_phi, lam_pi, ctx.tangent)
            grad_a = dlda.to(dtype=dtype, device=device).reshape(shape)
        else:
            grid.adjoint(n, lam_phi, lam_pi, gseries, None, project_initial=True, spin=False)
        ctx.grid = None
        ctx.ckpts = None
        grid.close()
        return lam_phi, lam_pi, grad_a, None, None, None, None, None, None


def evolve(phi0, pi0, a, cfg, n_steps, checkpoint_every=100, overlap=True, tangent=True, spin="forward"):
    """Extraction series of an n-step evolution, differentiable in phi0, pi0 and a."""
    if not torch.is_tensor(a):
        a = torch.tensor(float(a), dtype=torch.float64, device=phi0.device)
    return TeukEvolve.apply(phi0, pi0, a, cfg, n_steps, checkpoint_every, overlap, tangent, spin)
