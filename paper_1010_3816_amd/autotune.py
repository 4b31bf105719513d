"""Launch-shape autotuner for the step kernels.

The paper's only per-device tuning knob was OpenCL's local_work_size
(Sec. 4); here the knobs are the theta rows per wavefront tile, the
wavefronts per workgroup, on small grids the steps per launch of the block
pass (0: the sweeps) and, for batched launches, the number of workgroups
of the persistent launch.  Candidates are timed with HIP events on the
grid's own stream (median of three windows), the fastest is applied (for a
single grid only if it beats the library's default by a margin), and the
choice is cached in a JSON
file keyed by device and problem shape ($TEUK_TUNE_CACHE, default
~/.cache/paper_1010_3816_amd/launch.json).  Results of the kernels do not
depend on the launch shape, only their speed does.

Timing advances the state of the grid or batch: tune before setting the
initial data, or set it again afterwards.
"""
import json
import os

from . import binding

GRID_ROWS = (1, 2, 4, 8, 12, 16, 24, 32, 48, 64)
GRID_WAVES = (1, 2, 4, 8)
BATCH_ROWS = (8, 16, 32, 64, 128)
BATCH_WAVES = (1, 2, 4)


def _cache_path():
    return os.environ.get("TEUK_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_1010_3816_amd", "launch.json"))


def _load_cache():
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(key, value):
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        cache = _load_cache()
        cache[key] = value
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home only loses the cache


def _device_key(torch, device):
    p = torch.cuda.get_device_properties(device)
    return f"{getattr(p, 'gcnArchName', p.name)}/{p.multi_processor_count}cu"


def _time(torch, stream, fn, steps, reps=3):
    """Median over `reps` windows of `steps` steps (ms per step), after a
    short warm-up."""
    fn(2)
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn(steps)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) / steps)
    return sorted(times)[len(times) // 2]


def round_rows(nr, ntheta, cus, strip_cols=60, waves_per_simd=2, rounds=(1, 2, 3, 4), lo=1, hi=128):
    """Tile heights that cut each strip into as many tiles as fill k whole
    rounds of the device's resident wavefronts (k in `rounds`): a partly
    filled last round leaves SIMDs idle."""
    strips = -(-nr // strip_cols)
    slots = cus * 4 * waves_per_simd
    out = set()
    for k in rounds:
        chunks = k * slots // strips
        if chunks >= 1:
            r = -(-ntheta // chunks)
            if lo <= r <= hi:
                out.add(min(r, ntheta))
    return sorted(out)


def block_candidates(nr, ntheta, cus, lo=4):
    """(steps, cols) launches of the block pass worth timing on a grid (empty
    when the pass does not apply): workgroups of up to 256, 512 or 1024
    threads (at most 64 columns), from `lo` steps up to the most whose
    workgroups, one per CU, fit the device in one round."""
    if ntheta > 64:
        return []
    out = []
    for c in sorted({min(64, t // ntheta) for t in (256, 512, 1024)}):
        out += [(k, c) for k in range(lo, (c - 2) // 2 + 1) if -(-nr // (c - 2 * k)) <= cus]
    return out


def tune_grid(grid, rows=None, waves=GRID_WAVES, steps=20, use_cache=True, margin=0.02, blocks=None):
    """Pick the launch of a TeukGrid: (rows_per_tile, waves_per_block) of the
    sweeps and, on grids the block pass takes, its (steps, cols) launch
    (steps 0: the sweeps); returns {"rows": r, "waves": w, "block": k,
    "cols": c, "ms": t, "table": [...]}.  rows=None: GRID_ROWS and the
    heights of round_rows; blocks=None: block_candidates.  The library's
    default launch is kept unless a candidate is faster by more than
    `margin` (a fraction): run to run spread on the device is a few per cent,
    and the default is the round-filling shape."""
    torch = grid.torch
    key = f"grid|{_device_key(torch, grid.device)}|{grid.nr}x{grid.ntheta}"
    if use_cache:
        hit = _load_cache().get(key)
        if hit:
            grid.set_tile(min(hit["rows"], grid.ntheta), hit["waves"])
            grid.set_block_launch(hit.get("block", 0), hit.get("cols", 0))
            return dict(hit, cached=True)
    cus = torch.cuda.get_device_properties(grid.device).multi_processor_count
    if rows is None:
        rows = tuple(GRID_ROWS) + tuple(round_rows(grid.nr, grid.ntheta, cus))
    if blocks is None:
        blocks = block_candidates(grid.nr, grid.ntheta, cus)
    default = grid.tile() + grid.block_launch()
    table = []

    def timed(r, w, k, c):
        grid.set_tile(r, w)
        grid.set_block_launch(k, c)
        ms = _time(torch, grid.stream, lambda n: binding.teuk_step_n(grid.handle, n, None), steps)
        table.append({"rows": r, "waves": w, "block": k, "cols": c, "ms": ms})

    cands = {(min(r, grid.ntheta), w, 0, default[3]) for r in rows for w in waves}
    cands |= {default[:2] + (k, c) for k, c in blocks} | {default}
    for c in sorted(cands):
        timed(*c)
    best = min(table, key=lambda e: e["ms"])
    dflt = next(e for e in table if (e["rows"], e["waves"], e["block"], e["cols"]) == default)
    if dflt["ms"] <= best["ms"] * (1.0 + margin):
        best = dflt
    grid.set_tile(best["rows"], best["waves"])
    grid.set_block_launch(best["block"], best["cols"])
    out = {k: best[k] for k in ("rows", "waves", "block", "cols", "ms")}
    if use_cache:
        _store_cache(key, dict(out))
    out["table"] = table
    return out


def tune_batch(batch, rows=BATCH_ROWS, waves=BATCH_WAVES, blocks_per_cu=(1, 2, 4, 8), steps=10, use_cache=True):
    """Pick (rows_per_tile, waves_per_block, n_blocks) for a TeukBatch."""
    torch = batch.torch
    shapes = ",".join(f"{m['nr']}x{m['ntheta']}" for m in batch.members)
    import hashlib

    key = f"batch|{_device_key(torch, batch.device)}|{hashlib.sha256(shapes.encode()).hexdigest()[:16]}"
    if use_cache:
        hit = _load_cache().get(key)
        if hit:
            batch.set_launch(hit["rows"], hit["waves"], hit["blocks"])
            return dict(hit, cached=True)
    cus = torch.cuda.get_device_properties(batch.device).multi_processor_count
    table = []
    for r in rows:
        for w in waves:
            for k in blocks_per_cu:
                nb = max(1, cus * 4 * k // w)  # k wavefronts per SIMD
                batch.set_launch(r, w, nb)
                ms = _time(torch, batch.stream, batch.step, steps)
                table.append({"rows": r, "waves": w, "blocks": nb, "ms": ms})
    best = min(table, key=lambda e: e["ms"])
    batch.set_launch(best["rows"], best["waves"], best["blocks"])
    out = {"rows": best["rows"], "waves": best["waves"], "blocks": best["blocks"], "ms": best["ms"], "table": table}
    if use_cache:
        _store_cache(key, {"rows": best["rows"], "waves": best["waves"], "blocks": best["blocks"], "ms": best["ms"]})
    return out
