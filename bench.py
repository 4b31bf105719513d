"""Throughput benchmark of the fused Lax-Wendroff step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

One "step" is one Lax-Wendroff time step (Eqs. (lw1)-(lw2) of
arXiv:1010.3816 with the boundary updates) of the whole grid, launched
through the C ABI (teuk_step_n).  The default workload is the 25600 x 512
Kerr a = 0.99 grid (13.1 M points, 419 MB per state copy): it does not fit
in the 256 MB Infinity Cache, so HBM traffic is real.  The state is resident
in HBM before the timed region starts.  The library advances pairs of steps
in one pass (temporal blocking); the launch shape is autotuned first.

Prints one JSON line.  `value` is grid-point updates per second (one update
= one (r*, theta) point advanced one full step) over exactly the timed steps.
`roofline` describes the dominant kernel, the two-step pass: it moves 64
algorithmic bytes per point per pass (Phi, Pi read and written once,
complex128), i.e. 32 B per update, against HBM (`bound` "hbm", 8 TB/s), with
its FP64 rate and vector-instruction issue rate beside it, and the rates of
two plain copies (torch's and the library's own) for reference.  `repeats` are
five more windows as long as the timed one, `sustained` a window of 2000
steps (the device's steady state; short windows after an idle period run
slower while the clocks come up).  `c1` and `c2` are the 400 x 32 and
6400 x 256 workloads for all their steps with their extraction points, in
the library's default launch (the small-grid block pass on 400 x 32);
`batched` the 64-member uneven batch in one persistent launch per pass and
its ratio to `value`; `waveform` nine modes of one problem and their sum;
`adjoint` a waveform-loss gradient with respect to the initial data and the
spin on the 6400 x 256 grid: `ratio` = (forward + backward - plain
forward) / plain forward by the default route (the spin derivative carried
forward), and the checkpointed adjoint's routes beside it.  `source` is the
inhomogeneous variant (a localised source f(t) g(r*, theta) in the Pi
equation) on the default workload in the timed run's tile, 48 algorithmic
bytes per update, and its ratio to `value`.  `cpu_baseline` times
the CPU oracle (test infrastructure, plain C + OpenMP) on a bounded number of
steps of the same grid.
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FP64 grid-point updates/s + % HBM roofline; adjoint/forward time ratio"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
BYTES_PER_POINT_PASS = 64   # Phi, Pi read and written once per pass (complex128)
# the inhomogeneous variant at two steps a pass: the state's 64 B and the
# source profile's 32 B (g at the column and the half point) per point and pass
SOURCE_BYTES_PER_UPDATE = (BYTES_PER_POINT_PASS + 32) / 2
FLOPS_PER_UPDATE = {1: 230, 2: 192}  # FP64 flops per point and step, single-step and two-step kernels
VALU_PER_UPDATE = {1: 217, 2: 180}   # vector ALU instructions per point and step (from the SQ counters)
# vector instruction issue peak: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 instruction per 4 cycles per SIMD
VALU_PEAK_T = 256 * 4 * 2.4e9 * 64 / 4 / 1e12
KERNEL_SRCS = [os.path.join(ROOT, "paper_1010_3816_amd", "csrc", f)
               for f in ("lw_kernels.hip", "device_common.hpp", "internal.hpp")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "lw_step_kerr_a0.99_25600x512_traffic.txt")


def _code_only(text):
    """Source text without comments and with whitespace collapsed (string
    literals in these sources hold no comment markers)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash():
    """Hash of the code (comments and layout ignored) of the sources the step
    kernel is compiled from."""
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload, spp):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, if it was taken on this workload and kernel
    with the current kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if (kv.get("kernel_source_sha256") != kernel_source_hash() or kv.get("workload") != workload
            or kv.get("steps_per_launch") != str(spp)):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_bandwidth(torch, nbytes=1 << 30, reps=10):
    """Read + write rate (GB/s) of a plain device-to-device copy of nbytes
    (torch's copy_): what the device's HBM sustains for a pure stream, the
    practical ceiling beside the 8 TB/s peak."""
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    return 2 * nbytes / s / 1e9


def library_copy_bandwidth(torch, g, phi0, pi0, reps=10):
    """Read + write rate (GB/s) of the library's own plain copy kernel: the
    import of initial data into the grid's state (teuk_set_initial_data: per
    field, ntheta x (nr - 2) values read and ntheta x pitch written), timed on
    the grid's stream.  A second reference beside torch's copy, which streams
    more slowly on this device."""
    nr, nth = g.nr, g.ntheta
    pitch = (nr + 7) // 8 * 8
    moved = 2 * 16 * (nth * (nr - 2) + nth * pitch)
    g.set_initial_data(phi0, pi0)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(g.stream)
    for _ in range(reps):
        g.set_initial_data(phi0, pi0)
    e1.record(g.stream)
    torch.cuda.synchronize()
    return moved / (e0.elapsed_time(e1) / 1e3 / reps) / 1e9


def cpu_baseline(w, target_seconds=10.0, single_seconds=3.0):
    """The oracle as it stands, on the same grid, timed over whole steps
    until at least `target_seconds` have passed on all host threads, then
    `single_seconds` on one thread."""
    import numpy as np

    import oracle
    from paper_1010_3816_amd import inputs

    o = oracle.OracleGrid(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["dt"])
    phi, pi = inputs.initial_data(w)
    phi, pi = o.project(phi, pi)
    pts = w["nr"] * w["ntheta"]

    def timed(seconds):
        nonlocal phi, pi
        t0 = time.perf_counter()
        phi, pi = o.step(phi, pi, 1)
        one = time.perf_counter() - t0
        chunk = max(1, int(1.0 / max(one, 1e-6)))
        n, el = 0, 0.0
        t0 = time.perf_counter()
        while el < seconds:
            phi, pi = o.step(phi, pi, chunk)
            n += chunk
            el = time.perf_counter() - t0
        assert np.isfinite(phi).all()
        return pts * n / el, f"{n} steps of the full {w['nr']}x{w['ntheta']} grid ({el:.1f} s), after 1 untimed step"

    threads = oracle.num_threads()
    value, sample = timed(target_seconds)
    oracle.set_num_threads(1)
    try:
        value1, sample1 = timed(single_seconds)
    finally:
        oracle.set_num_threads(threads)
    return {"value": value, "unit": "grid-point updates/s", "cores": threads, "kind": "oracle", "sample": sample,
            "single_thread": {"value": value1, "cores": 1, "sample": sample1}}


def waveform_leg(n_samples=500, sample_every=2):
    """The field from its modes: nine modes m = -4..4 (s = -2, a = 0.7) on the
    6400 x 256 grid, advanced as one batch and sampled at four observers every
    `sample_every` steps (one launch for all modes and observers), then summed
    into Psi = r^3 sum_m e^{i m phi} Phi_m.  Member grid-point updates/s over
    the sampled evolution, the share of that time spent sampling, and the
    assembly time."""
    import torch

    from paper_1010_3816_amd import inputs
    from paper_1010_3816_amd.waveform import ModeSet

    a, s, nr, nth, r0, r1 = 0.7, -2, 6400, 256, -100.0, 600.0
    modes = list(range(-4, 5))
    steps = n_samples * sample_every
    dr = (r1 - r0) / (nr - 1)
    dt = min(inputs.stable_dt(dr, nth, m, s, steps) for m in modes)
    obs = [(500.0, math.pi / 2, 0.0), (500.0, math.pi / 2, math.pi / 3), (500.0, math.pi / 4, 0.0),
           (300.0, 2.0, 1.0)]
    W = ModeSet(a, s, modes, nr, nth, r0, r1, dt, obs)
    for m in modes:
        p, q = inputs.gaussian_pulse(nr, nth, r0, r1, 12.0, 4.0, "regular", m, s)
        W.set_initial_data(m, torch.from_numpy(p).cuda(), torch.from_numpy(q).cuda())
    W.evolve(4, sample_every)  # warm-up (captures the batch's graph)
    stream = W.batch.stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    samples = W.evolve(n_samples, sample_every)
    ev[1].record(stream)
    psi = W.assemble(samples)
    ev[2].record(stream)
    ev[3].record(stream)
    W.batch.step(steps)  # the same steps without sampling
    ev[4].record(stream)
    torch.cuda.synchronize()
    ms_evolve, ms_assemble, ms_plain = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[3].elapsed_time(ev[4])
    assert bool(torch.isfinite(psi.real).all()) and bool(torch.isfinite(psi.imag).all()), "Psi became non-finite"
    pts = W.batch.total_points()
    W.close()
    return {"modes": len(modes), "m": [modes[0], modes[-1]], "grid": f"{nr}x{nth}", "points_per_step": pts,
            "steps": steps, "sample_every": sample_every, "observers": len(obs),
            "value": pts * steps / (ms_evolve * 1e-3), "unit": "member grid-point updates/s",
            "ms_per_step": ms_evolve / steps, "sampling_share": 1.0 - ms_plain / ms_evolve,
            "assemble_ms": ms_assemble, "samples": n_samples}


def batched_leg(steps=200, launch=None):
    """64 uneven evolutions in one persistent launch per step (autotuned
    unless `launch` = (rows, waves_per_block, blocks) is given)."""
    import torch

    from paper_1010_3816_amd import autotune, binding, inputs

    mbs = inputs.batch_members()
    b = binding.TeukBatch(mbs)
    if launch is None:
        tune = autotune.tune_batch(b, use_cache=False)
    else:
        b.set_launch(*launch)
        tune = {"rows": launch[0], "waves": launch[1], "blocks": launch[2]}
    for k, mb in enumerate(mbs):
        p, q = inputs.initial_data(mb)
        b.set_initial_data(k, torch.from_numpy(p).cuda(), torch.from_numpy(q).cuda())
    b.step(10)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(b.stream)
    b.step(steps)
    e1.record(b.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    pts = b.total_points()
    out = {"value": pts / (ms * 1e-3), "unit": "member grid-point updates/s", "members": len(mbs),
           "points_per_step": pts, "steps": steps, "ms_per_step": ms,
           "launch": {"rows": tune["rows"], "waves_per_block": tune["waves"], "blocks": tune["blocks"]}}
    b.close()
    return out


def workload_leg(name):
    """A standard workload for all its steps from its own initial data, with
    its extraction points, in the library's default launch: updates/s and ms
    per step over the whole run (HIP events on the grid's stream)."""
    import torch

    from paper_1010_3816_amd import binding, inputs

    w = inputs.workload(name)
    g = binding.TeukGrid(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["dt"],
                         extract_rstar=w["extract_rstar"], extract_theta=w["extract_theta"])
    phi0, pi0 = (torch.from_numpy(x).cuda() for x in inputs.initial_data(w))
    n = w["steps"]
    series = torch.empty((n, g.n_extract), dtype=torch.complex128, device="cuda")
    g.set_initial_data(phi0, pi0)
    binding.teuk_step_n(g.handle, min(n, 200), series)  # warm-up
    g.set_initial_data(phi0, pi0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(g.stream)
    binding.teuk_step_n(g.handle, n, series)
    e1.record(g.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    assert g.check_finite(), "state became non-finite"
    rows, wpb = g.tile()
    out = {"workload": name, "steps": n, "n_extract": g.n_extract, "ms_per_step": ms / n,
           "value": w["nr"] * w["ntheta"] * n / (ms * 1e-3), "unit": "grid-point updates/s",
           "tile_rows": rows, "waves_per_block": wpb,
           # small grids: steps per launch of the block pass (0: the sweeps, with the tile above)
           # and the columns a workgroup holds
           "block_steps": g.block_launch()[0], "block_cols": g.block_launch()[1]}
    g.close()
    return out


def source_leg(name="kerr_a0.99_25600x512", steps=1000, tile=None):
    """The inhomogeneous variant: a standard workload's pulse plus a
    localised source f(t) g(r*, theta) (a blob at r* = centre + 20 on the
    equator, f = 50 exp(0.4 i t)), `steps` steps of teuk_step_n_source in the
    tile `tile` (rows, waves_per_block), timed with HIP events on the grid's
    stream.  Algorithmic bytes: the state's 64 B per point per pass of two
    steps and the profile's 32 B (g at the column and at the half point, read
    once a pass), 48 B per update."""
    import torch

    from paper_1010_3816_amd import binding, inputs

    w = inputs.workload(name)
    g = binding.TeukGrid(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["dt"])
    if tile is not None:
        g.set_tile(*tile)
    gi, gh = inputs.localised_source(w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["center"] + 20.0)
    g.set_source(torch.from_numpy(gi).cuda(), torch.from_numpy(gh).cuda())
    del gi, gh
    phi0, pi0 = (torch.from_numpy(x).cuda() for x in inputs.initial_data(w))
    f = inputs.oscillating_factors(steps, w["dt"])
    g.set_initial_data(phi0, pi0)
    g.step_source(f[: min(steps, 100)], series=False)  # warm-up
    g.set_initial_data(phi0, pi0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(g.stream)
    g.step_source(f, series=False)
    e1.record(g.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    assert g.check_finite(), "state became non-finite"
    ups = w["nr"] * w["ntheta"] * steps / (ms * 1e-3)
    rows, wpb = g.tile()
    out = {"workload": name, "source": "localised blob at r* = centre + 20, theta = pi/2; f = 50 exp(0.4 i t)",
           "steps": steps, "ms_per_step": ms / steps, "value": ups, "unit": "grid-point updates/s",
           "steps_per_pass": g.steps_per_pass(), "bytes_per_update": SOURCE_BYTES_PER_UPDATE,
           "hbm_frac": SOURCE_BYTES_PER_UPDATE * ups / 1e9 / HBM_PEAK_GBS, "tile_rows": rows, "waves_per_block": wpb}
    g.close()
    return out


def adjoint_leg(n_steps=None, checkpoint_every=None):
    """Loss and gradients of the waveform misfit on the adjoint workload:
    6400 x 256, a = 0.7, 8000 steps, target = series of the perturbed run
    (a + 0.01, centre + 0.5), gradients with respect to the initial data and
    the spin.  Routes for the spin: carried forward (the default: the
    forward pass advances du/da too, the backward is one cotangent sweep),
    and the checkpointed adjoint (a checkpoint every 100 steps; recompute of
    the step tangents or of the states).  plain_forward_ms: the same loss
    without gradients.  ratio = (forward + backward - plain forward) /
    plain forward, the gradient's cost beyond the forward pass in forward
    passes (for the checkpointed route, whose forward is the plain one plus
    checkpoint copies, about backward / forward)."""
    import torch

    from paper_1010_3816_amd import inputs
    from paper_1010_3816_amd.autograd import evolve

    w = inputs.workload("adjoint_a0.7_6400x256")
    n_steps = n_steps or w["steps"]
    checkpoint_every = checkpoint_every or w["checkpoint_every"]
    cfg = {k: w[k] for k in ("s", "m", "nr", "ntheta", "rstar_min", "rstar_max", "dt", "extract_rstar",
                             "extract_theta")}
    wt = inputs.adjoint_target(w)
    with torch.no_grad():
        pt, qt = (torch.from_numpy(x).cuda() for x in inputs.initial_data(wt))
        target = evolve(pt, qt, wt["a"], cfg, n_steps, n_steps).clone()
        del pt, qt
    p0, q0 = inputs.initial_data(w)
    P = torch.from_numpy(p0).cuda().requires_grad_(True)
    Q = torch.from_numpy(q0).cuda().requires_grad_(True)
    A = torch.tensor(w["a"], dtype=torch.float64, device="cuda", requires_grad=True)

    def timed(a, **kw):
        times = []
        for _ in range(2):  # the first pass warms up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ser = evolve(P, Q, a, cfg, n_steps, checkpoint_every, **kw)
            L = ((ser - target).abs() ** 2).sum()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            L.backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            times.append((t1 - t0, t2 - t1))
            dlda = float(A.grad) if a is A else None
            P.grad = Q.grad = A.grad = None
        return times[-1][0] * 1e3, times[-1][1] * 1e3, float(L.detach()), dlda

    # the plain forward: the same loss with no gradient at all
    plain = []
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.no_grad():
            L = ((evolve(P.detach(), Q.detach(), A.detach(), cfg, n_steps, checkpoint_every) - target).abs() ** 2).sum()
        torch.cuda.synchronize()
        plain.append((time.perf_counter() - t0) * 1e3)
    plain_ms = plain[-1]

    def route(fwd, bwd, loss, dlda, name):
        return {"route": name, "forward_ms": fwd, "backward_ms": bwd, "backward_over_forward": bwd / fwd,
                "ratio": (fwd + bwd - plain_ms) / plain_ms, "loss": loss, "dL_da": dlda}

    fw = route(*timed(A, spin="forward"), "spin derivative carried forward")
    rt = route(*timed(A, spin="reverse", tangent=True), "checkpointed adjoint, stored step tangents")
    rs = route(*timed(A, spin="reverse", tangent=False), "checkpointed adjoint, stored states")
    # gradients with respect to the initial data only: one cotangent sweep
    f0, b0, _, _ = timed(A.detach())
    return {"workload": "adjoint_a0.7_6400x256", "steps": n_steps, "checkpoint_every": checkpoint_every,
            "extract": [w["extract_rstar"][0], w["extract_theta"][0]], "loss": fw["loss"], "dL_da": fw["dL_da"],
            "plain_forward_ms": plain_ms, "forward_ms": fw["forward_ms"], "backward_ms": fw["backward_ms"],
            "ratio": fw["ratio"],
            "ratio_definition": "(forward + backward - plain forward) / plain forward, spin carried forward",
            "route": fw["route"], "reverse_tangent_route": rt, "reverse_state_route": rs,
            "initial_data_only": {"forward_ms": f0, "backward_ms": b0, "backward_over_forward": b0 / f0}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="kerr_a0.99_25600x512")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched and adjoint legs")
    ap.add_argument("--only", choices=["batched", "adjoint", "waveform", "c1", "c2", "source"],
                    help="run only this leg and print its JSON object (for profiling)")
    ap.add_argument("--batch-launch", default=None,
                    help="rows,waves_per_block,blocks for the batched leg (default: autotune)")
    ap.add_argument("--tile", default=None,
                    help="rows,waves_per_block of the step kernel (default: autotune)")
    ap.add_argument("--steps-per-pass", type=int, choices=[1, 2], default=None,
                    help="force one or two steps per kernel pass (default: the library's, two)")
    ap.add_argument("--adjoint-steps", type=int, default=None,
                    help="steps of the adjoint leg (default: the workload's 8000; fewer for profiling)")
    ap.add_argument("--calibrate", action="store_true",
                    help="also run a plain 1 GiB streaming kernel (for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(independent grids and m-modes shard across GPUs without communication)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1010_3816_amd import autotune, binding, inputs

    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    launch = tuple(int(x) for x in args.batch_launch.split(",")) if args.batch_launch else None
    if args.only == "batched":
        print(json.dumps(batched_leg(launch=launch)), flush=True)
        return
    if args.only == "waveform":
        print(json.dumps(waveform_leg()), flush=True)
        return
    if args.only == "adjoint":
        print(json.dumps(adjoint_leg(n_steps=args.adjoint_steps)), flush=True)
        return
    if args.only == "source":
        print(json.dumps(source_leg(tile=tuple(int(x) for x in args.tile.split(",")) if args.tile else None)),
              flush=True)
        return
    if args.only in ("c1", "c2"):
        name = {"c1": "schwarzschild_400x32", "c2": "kerr_a0.9_6400x256"}[args.only]
        print(json.dumps(workload_leg(name)), flush=True)
        return
    w = inputs.workload(args.workload)
    g = binding.TeukGrid(w["a"], w["s"], w["m"], w["nr"], w["ntheta"], w["rstar_min"], w["rstar_max"], w["dt"],
                         extract_rstar=w["extract_rstar"], extract_theta=w["extract_theta"])
    if args.steps_per_pass:
        g.set_steps_per_pass(args.steps_per_pass)
    spp = g.steps_per_pass()
    # The initial data are made and moved to the device first; the launch
    # shape is tuned on the grid after that, so the device works up to the
    # warm-up and the timed region (an idle device lowers its clocks, and
    # short windows then run slower).  The timed run starts from the
    # workload's data again.
    phi0, pi0 = (torch.from_numpy(x).cuda() for x in inputs.initial_data(w))
    g.set_initial_data(phi0, pi0)
    n_series = max(args.steps, args.warmup, 2000, 1)
    series = torch.empty((n_series, max(g.n_extract, 1)), dtype=torch.complex128, device="cuda")
    stream = g.stream

    def run(n):
        binding.teuk_step_n(g.handle, n, series if g.n_extract else None)

    if args.tile:
        g.set_tile(*(int(x) for x in args.tile.split(",")))
    else:
        autotune.tune_grid(g, waves=(1, 2, 4), steps=50, use_cache=False)
    g.set_initial_data(phi0, pi0)
    run(args.warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    run(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    assert g.check_finite(), "state became non-finite"
    # run-to-run spread: five more windows as long as the timed one, then the
    # steady state over 2000 steps (outside the timed region)
    n_rep = args.steps
    reps = []
    for _ in range(5):
        a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a0.record(stream)
        run(n_rep)
        a1.record(stream)
        torch.cuda.synchronize()
        reps.append(w["nr"] * w["ntheta"] * n_rep / (a0.elapsed_time(a1) * 1e-3))
    a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a0.record(stream)
    run(2000)
    a1.record(stream)
    torch.cuda.synchronize()
    ms_sus = a0.elapsed_time(a1) / 2000
    assert g.check_finite(), "state became non-finite"

    pts = w["nr"] * w["ntheta"]
    ms_step = ms / args.steps
    ups = pts / (ms_step * 1e-3)
    # per launch of the dominant kernel (spp steps per launch)
    launch_s = spp * ms_step * 1e-3
    hbm_gbs = BYTES_PER_POINT_PASS * pts / launch_s / 1e9
    tflops = FLOPS_PER_UPDATE[spp] * spp * pts / launch_s / 1e12
    traffic = measured_traffic(args.workload, spp)
    copy_torch = copy_bandwidth(torch)
    copy_lib = library_copy_bandwidth(torch, g, phi0, pi0)
    copy_gbs = max(copy_torch, copy_lib)
    traffic_gbs = traffic / launch_s / 1e9 if traffic else None
    rows, wpb = g.tile()
    valu = VALU_PER_UPDATE[spp] * spp * pts / launch_s / 1e12
    # Both passes are bound by HBM: the one-step pass streams its 64 B per
    # update at a plain copy's rate; the two-step pass moves its measured
    # traffic (halo rows and strip overlap on top of 32 B per update) at
    # nearly that rate, with the vector ALUs busy about two thirds of the time.
    roof = {"bound": "hbm", "achieved": hbm_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": hbm_gbs / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "lw_step2_kernel" if spp == 2 else "lw_step_kernel", "steps_per_launch": spp,
            "bytes_per_update": BYTES_PER_POINT_PASS / spp,
            # measured HBM traffic per launch over the launch time, and a plain copy's rate on this
            # device: the faster of torch's copy and the library's own import copy
            "traffic_achieved": traffic_gbs, "copy_achieved": copy_gbs,
            "copy_torch": copy_torch, "copy_library": copy_lib,
            "traffic_over_copy": traffic_gbs / copy_gbs if traffic_gbs else None,
            "achieved_over_copy": hbm_gbs / copy_gbs,
            # the one-step-per-pass bound (64 B per update at 8 TB/s) and this run against it
            "one_step_bound_updates_per_s": HBM_PEAK_GBS * 1e9 / BYTES_PER_POINT_PASS,
            "value_over_one_step_bound": ups / (HBM_PEAK_GBS * 1e9 / BYTES_PER_POINT_PASS),
            "fp64": {"achieved": tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": tflops / FP64_PEAK_TFLOPS, "flops_per_update": FLOPS_PER_UPDATE[spp]},
            "valu_issue": {"achieved": valu, "peak": VALU_PEAK_T, "unit": "T lane-instructions/s",
                           "frac": valu / VALU_PEAK_T, "instructions_per_update": VALU_PER_UPDATE[spp]}}

    if args.calibrate:
        n = 1 << 27  # 1 GiB of float64
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b

    out = {
        "metric": METRIC,
        "value": ups,
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "nr": w["nr"], "ntheta": w["ntheta"], "a": w["a"], "s": w["s"],
                   "m": w["m"], "rstar": [w["rstar_min"], w["rstar_max"]], "dt": w["dt"],
                   "n_extract": g.n_extract, "steps_per_pass": spp, "tile_rows": rows, "waves_per_block": wpb},
        "roofline": roof,
        "wall_s_timed_region": wall,
        "repeats": {"windows": 5, "steps_each": n_rep, "median": sorted(reps)[2], "min": min(reps), "max": max(reps)},
        "sustained": {"steps": 2000, "ms_per_step": ms_sus,
                      "value": w["nr"] * w["ntheta"] / (ms_sus * 1e-3),
                      "roofline_frac": BYTES_PER_POINT_PASS * w["nr"] * w["ntheta"] / (spp * ms_sus * 1e-3) / 1e9
                      / HBM_PEAK_GBS},
    }
    g.close()
    if not args.no_extras:
        out["c1"] = workload_leg("schwarzschild_400x32")
        out["c2"] = workload_leg("kerr_a0.9_6400x256")
        bl = batched_leg(launch=launch)
        bl["ratio_to_single"] = bl["value"] / ups
        out["batched"] = bl
        wl = waveform_leg()
        wl["ratio_to_single"] = wl["value"] / ups
        out["waveform"] = wl
        out["adjoint"] = adjoint_leg()
        sl = source_leg(args.workload, tile=(rows, wpb))
        sl["ratio_to_homogeneous"] = sl["value"] / ups
        out["source"] = sl
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
