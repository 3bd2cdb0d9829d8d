"""Tile-plan autotuner for the cell-sorted particle passes.

The tiled passes have four knobs (pic_config_t): the tile edge in cells
(`tile_cells`), the particles per workgroup (`chunk`), the steps between
re-sorts (`sort_interval`) and whether step() fuses the gather/push with the
next deposit (PIC_FLAG_UNFUSED_STEP).  Their
best values depend on the grid, the particles per cell and the particle
precision, so they are measured: every candidate plan runs a few steps of the
caller's own workload (warm-up steps first, so the first sort and the graph
capture stay out of the timing), timed with HIP events on the context's
stream, and the fastest plan wins.  Results are cached in a JSON file keyed
by the workload's shape and the device name.

    plan = tune(key, make_cfgs, load)   # {"tile_cells", "chunk", "unfused", "sort_interval"}
    cfgs = apply(make_cfgs(), plan)

`make_cfgs()` returns the pic_config_t list of the workload (one entry for a
plain run, one per instance for an ensemble) and `load(ctx)` puts the
particles into a fresh context.
"""

import json
import os

import torch

from . import pic

# candidate plans: tile edge x chunk x fused/unfused x sort interval (0: the
# library's worst-case interval, slack / (c dt / dx); longer intervals stay
# correct -- particles that leave their window take the global path -- and pay
# off when particles are slower than c)
CANDIDATES = [dict(tile_cells=t, chunk=c, unfused=u, sort_interval=si)
              for t in (8, 16) for c in (512, 1024, 2048, 4096) for u in (False, True) for si in (0, 12)]
KNOBS = ("tile_cells", "chunk", "unfused", "sort_interval")


def default_cache_path():
    base = os.environ.get("PIC_AUTOTUNE_CACHE")
    if base:
        return base
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2410_18414_amd", "autotune.json")


def apply(cfgs, plan):
    """Copies of the configs with the plan's knobs set."""
    out = []
    for c in cfgs:
        d = pic.ConfigStruct()
        ctypes_copy(d, c)
        d.tile_cells = min(plan["tile_cells"], c.nx, c.ny)
        d.chunk = plan["chunk"]
        d.sort_interval = plan.get("sort_interval", 0)
        d.flags = (c.flags & ~pic.FLAG_UNFUSED_STEP) | (pic.FLAG_UNFUSED_STEP if plan["unfused"] else 0)
        out.append(d)
    return out


def ctypes_copy(dst, src):
    for name, _ in pic.ConfigStruct._fields_:
        setattr(dst, name, getattr(src, name))


def measure(cfgs, load, steps=24, warmup=6):
    """ms per step of one plan (the context is built, loaded and dropped).
    The warm-up spans at least one graph period plus a step, so the one-time
    graph capture is not timed."""
    ctx = pic.Context(cfgs if len(cfgs) > 1 else cfgs[0])
    try:
        load(ctx)
        run = pic.step_batched if len(cfgs) > 1 else pic.step
        run(ctx, max(warmup, pic.graph_period(ctx) + 1))
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(ctx.stream)
        run(ctx, steps)
        b.record(ctx.stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps
    finally:
        ctx.close()


def tune(key, make_cfgs, load, candidates=None, steps=24, warmup=6, cache_path=None, refresh=False):
    """Best plan for the workload `key` (measured once, then read from the cache)."""
    cache_path = cache_path or default_cache_path()
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    full_key = "%s|%s" % (dev, key)
    cache = {}
    if os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if not refresh and full_key in cache:
        return dict(cache[full_key]["best"], cached=True)
    results = []
    for cand in (candidates or CANDIDATES):
        ms = measure(apply(make_cfgs(), cand), load, steps=steps, warmup=warmup)
        results.append(dict(cand, ms_per_step=ms))
    best = min(results, key=lambda r: r["ms_per_step"])
    plan = {k: best[k] for k in KNOBS}
    cache[full_key] = dict(best=plan, results=results)
    try:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    except OSError:
        pass
    return dict(plan, cached=False, results=results)
