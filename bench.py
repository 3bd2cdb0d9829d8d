"""Throughput of the full PIC step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--repeats R] [--gpus 1] [--workload weibel512-dirk2]

One step = Algorithm 1 once over every particle: position update and current
deposit, FFT field solve (continuity + stepper update + spectral gradients),
gather and IAEM push (the libpic `step` entry point, gather/push of step n
fused with the deposit of step n+1).  Inputs are resident in HBM before the
timed regions; each of R timed regions of exactly K steps is bracketed by
device synchronisations, and the median region is reported.

The headline workload is the 512 x 512 grid with 256 particles per cell
(67,108,864 float32 particles, cubic splines, DIRK-2), the largest
single-GPU configuration.  Prints one JSON line with its particle-steps/s
value, a roofline entry for the dominant kernel (the fused
gather/push/deposit particle pass, timed with HIP events on the library's
stream), the same workload under CDF-2 and the 128 x 128 workload as
sections, the batched form (64-instance uneven ensemble, tile plan from the
autotuner) and the adjoint form (gradient through 20 float64 steps) against
the plain step, and the FP64 oracle timed on one host core on a bounded
sample of the headline workload.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s per full PIC step; batched and adjoint vs plain at 1e-10 rel"
HBM_PEAK_GBS = 8000.0

# name -> (workload name in paper_2410_18414_amd.workloads, overrides, label)
WORKLOADS = {
    "weibel128": ("weibel128", {}, "weibel-128x128-64ppc-cubic-bdf2-f32"),
    "weibel512-dirk2": ("weibel512", {}, "weibel-512x512-256ppc-cubic-dirk2-f32"),
    "weibel512-cdf2": ("weibel512", {"scheme": "cdf2"}, "weibel-512x512-256ppc-cubic-cdf2-f32"),
    "cloud32": ("cloud32", {}, "cloud-32x32-4ppc-quadratic-bdf1-f64"),
}


def particle_bytes(dtype):
    """Algorithmic HBM bytes per particle of the fused pass: read x, y, P(3),
    v^n(3), v^{n-1}(3); write x, y, Px, Py, v^{n+1}(3) (P_z is constant in 2-D)."""
    es = 4 if dtype == "f32" else 8
    return (11 + 7) * es


def grid_bytes(nx, ny, dtype):
    """Per launch: one read of the 11 gathered mesh fields (particle dtype) and
    one read-modify-write of the three float64 J planes."""
    es = 4 if dtype == "f32" else 8
    return nx * ny * (11 * es + 3 * 8 * 2)


def measured_traffic(tag):
    """HBM bytes per launch of the fused pass from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (profiles/traffic_<tag>.md), or None when
    there is none or the kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_%s.md" % tag)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        key, sep, val = line.strip().partition(": ")
        if sep and key in ("traffic_bytes_per_launch", "kernel_sources_sha256", "kernel_sources"):
            fields[key] = val.strip()
    if len(fields) != 3:
        return None
    h = hashlib.sha256()
    for src in fields["kernel_sources"].split():
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if h.hexdigest() != fields["kernel_sources_sha256"]:
        return None
    return int(fields["traffic_bytes_per_launch"])


def cpu_description():
    """The host CPU as /proc/cpuinfo names it (model string, vendor, family,
    model and stepping numbers, clock and cache of the first logical CPU) and
    the logical CPUs this process may run on."""
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if not line.strip():
                    break  # first logical CPU only
                key, _, val = line.partition(":")
                info[key.strip()] = val.strip()
    except OSError:
        pass
    keys = ("model name", "vendor_id", "cpu family", "model", "stepping", "cpu MHz", "cache size")
    desc = "; ".join("%s: %s" % (k, info[k]) for k in keys if k in info) or "unknown"
    return desc, len(os.sched_getaffinity(0))


def cpu_baseline(w, spec, nsub, nsteps):
    """The FP64 oracle (numpy) on a bounded sample of the same workload: its
    first `nsub` particles (uniformly placed, so the sample keeps the
    workload's spatial distribution at nsub / n of its density) on the full
    grid with the same stepper, `nsteps` complete steps, on ONE host core:
    the calling thread is pinned to one CPU and the BLAS/OpenMP pools are
    limited to one thread while the oracle runs."""
    from threadpoolctl import threadpool_limits

    from oracle import pic as opic
    nsub = min(nsub, len(w["x"]))
    p = opic.Params(w["nx"], w["ny"], w["lx"], w["ly"], spec["degree"], spec["scheme"], w["dt"],
                    q=w["q"], m=w["m"], bdf_order=spec["bdf_order"])
    x, y, P = w["x"][:nsub].copy(), w["y"][:nsub].copy(), w["P"][:nsub].copy()
    mask = os.sched_getaffinity(0)
    core = min(mask)
    os.sched_setaffinity(0, {core})
    try:
        with threadpool_limits(limits=1):
            s = opic.State(p, x, y, P)
            t0, c0 = time.perf_counter(), time.thread_time()
            s.step(nsteps)
            dt, cpu = time.perf_counter() - t0, time.thread_time() - c0
    finally:
        os.sched_setaffinity(0, mask)
    desc, ncpu = cpu_description()
    return dict(value=nsub * nsteps / dt, unit="particle-steps/s", cores=1, kind="oracle",
                sample="%d full %s steps of the first %d of the workload's %d particles on its full %dx%d grid "
                       "(numpy float64; one thread pinned to one core)"
                       % (nsteps, spec["scheme"], nsub, len(w["x"]), w["nx"], w["ny"]),
                seconds=round(dt, 2), thread_cpu_seconds=round(cpu, 2),
                cpu_model=desc, host_logical_cpus=ncpu)


def _events(stream):
    import torch
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    return a, b


def bench_batched(steps, warmup):
    """The 64-instance uneven ensemble (grids 32..256 per side, 4..64
    particles/cell, Maxwellian clouds, cubic, BDF-2, float32) as one context
    (step_batched: one launch per phase over all instances, graph-replayed),
    with the tile plan from the autotuner, against the same 64 instances run
    one after another as plain contexts with the same plan."""
    import torch
    from paper_2410_18414_amd import autotune, pic, workloads
    ws = workloads.ensemble()
    dev = torch.device("cuda:0")
    data = [(torch.as_tensor(w["x"], device=dev), torch.as_tensor(w["y"], device=dev),
             torch.as_tensor(np.ascontiguousarray(w["P"].T), device=dev)) for w in ws]
    total = sum(len(w["x"]) for w in ws)

    def make_cfgs():
        return [pic.make_config(w["nx"], w["ny"], w["lx"], w["ly"], w["dt"], degree=3, scheme="bdf",
                                bdf_order=2, dtype="f32", q=w["q"], m=w["m"], max_particles=len(w["x"]))
                for w in ws]

    def load(ctx):
        for i, (x, y, P) in enumerate(data):
            if pic.instance_count(ctx) > 1:
                pic.select_instance(ctx, i)
            pic.init_particles(ctx, x, y, P)

    plan = autotune.tune("ensemble64-draw4999-seeds4000-cubic-bdf2-f32", make_cfgs, load)
    cfgs = autotune.apply(make_cfgs(), plan)
    ctx = pic.Context(cfgs)
    load(ctx)
    pic.step_batched(ctx, max(warmup, pic.graph_period(ctx) + 1))
    a, b = _events(ctx.stream)
    torch.cuda.synchronize()
    a.record(ctx.stream)
    pic.step_batched(ctx, steps)
    b.record(ctx.stream)
    torch.cuda.synchronize()
    ms_b = a.elapsed_time(b) / steps
    ctx.close()
    del ctx
    # the same instances one after another, each its own context
    ms_p = 0.0
    for i, cfg in enumerate(cfgs):
        c = pic.Context(cfg)
        pic.init_particles(c, *data[i])
        pic.step(c, max(warmup, pic.graph_period(c) + 1))
        a, b = _events(c.stream)
        torch.cuda.synchronize()
        a.record(c.stream)
        pic.step(c, steps)
        b.record(c.stream)
        torch.cuda.synchronize()
        ms_p += a.elapsed_time(b) / steps
        c.close()
    return dict(workload="ensemble of 64 uneven Maxwellian clouds (grids 32..256 per side, 4..64 ppc, "
                         "cubic, BDF-2, f32)", instances=len(ws), particles=total, steps=steps,
                ms_per_step=round(ms_b, 5), value=round(total / (ms_b * 1e-3), 1),
                plain_ms_per_step=round(ms_p, 5), plain_value=round(total / (ms_p * 1e-3), 1),
                speedup_vs_plain=round(ms_p / ms_b, 3),
                tile_plan={k: plan[k] for k in autotune.KNOBS},
                tile_plan_cached=bool(plan.get("cached")))


def bench_batched_integer_sides(steps=20, warmup=6):
    """The uneven ensemble under the strict reading of its grid draw: 64
    Maxwellian clouds whose sides are uniform integers in [32, 256] (none a
    power of two here: mixed-radix FFTs, partial tiles, the generic tiled
    kernel), 4..64 particles/cell, cubic, BDF-2, float32, as one context with
    the autotuner's tile plan."""
    import torch
    from paper_2410_18414_amd import autotune, pic, workloads
    ws = workloads.ensemble(sizes=slice(32, 256))
    dev = torch.device("cuda:0")
    data = [(torch.as_tensor(w["x"], device=dev), torch.as_tensor(w["y"], device=dev),
             torch.as_tensor(np.ascontiguousarray(w["P"].T), device=dev)) for w in ws]
    total = sum(len(w["x"]) for w in ws)

    def make_cfgs():
        return [pic.make_config(w["nx"], w["ny"], w["lx"], w["ly"], w["dt"], degree=3, scheme="bdf", bdf_order=2,
                                dtype="f32", q=w["q"], m=w["m"], max_particles=len(w["x"])) for w in ws]

    def load(ctx):
        for i, (x, y, P) in enumerate(data):
            pic.select_instance(ctx, i)
            pic.init_particles(ctx, x, y, P)

    plan = autotune.tune("ensemble64-intsides32-256-draw4999-seeds4000-cubic-bdf2-f32", make_cfgs, load)
    ctx = pic.Context(autotune.apply(make_cfgs(), plan))
    load(ctx)
    pic.step_batched(ctx, max(warmup, pic.graph_period(ctx) + 1))
    a, b = _events(ctx.stream)
    torch.cuda.synchronize()
    a.record(ctx.stream)
    pic.step_batched(ctx, steps)
    b.record(ctx.stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    pow2 = sum(1 for w in ws if not (w["nx"] & (w["nx"] - 1) or w["ny"] & (w["ny"] - 1)))
    ctx.close()
    return dict(workload="ensemble of 64 Maxwellian clouds, sides uniform integers in [32, 256], 4..64 ppc, "
                         "cubic, BDF-2, f32", instances=len(ws), power_of_two_instances=pow2, particles=total,
                steps=steps, ms_per_step=round(ms, 5), value=round(total / (ms * 1e-3), 1),
                tile_plan={k: plan[k] for k in autotune.KNOBS}, tile_plan_cached=bool(plan.get("cached")))


def bench_naive(steps=20):
    """The paper's naive comparison (rho mapped with the spline instead of
    continuity) on the plain workload: its step rate, and the relative gauge
    and Gauss residuals after `steps` steps for both updates."""
    import torch
    from paper_2410_18414_amd import pic, workloads
    w = workloads.make("weibel128")
    n = len(w["x"])
    dev = torch.device("cuda:0")
    data = (torch.as_tensor(w["x"], device=dev), torch.as_tensor(w["y"], device=dev),
            torch.as_tensor(np.ascontiguousarray(w["P"].T), device=dev))
    out = dict(workload="weibel-128x128-64ppc-cubic-bdf2-f32, %d steps" % steps, particles=n, steps=steps)
    for name, flags in (("continuity", 0), ("naive", pic.FLAG_NAIVE_RHO)):
        cfg = pic.make_config(w["nx"], w["ny"], w["lx"], w["ly"], w["dt"], degree=3, scheme="bdf", bdf_order=2,
                              dtype="f32", q=w["q"], m=w["m"], max_particles=n, flags=flags)
        ctx = pic.Context(cfg)
        # warm-up (past the graph capture where the passes replay graphs), then
        # a fresh start timed over `steps` steps
        pic.init_particles(ctx, *data)
        pic.step(ctx, pic.graph_period(ctx) + 1)
        pic.init_particles(ctx, *data)
        a, b = _events(ctx.stream)
        torch.cuda.synchronize()
        a.record(ctx.stream)
        pic.step(ctx, steps)
        b.record(ctx.stream)
        torch.cuda.synchronize()
        d = pic.diagnostics(ctx)
        ms = a.elapsed_time(b) / steps
        out[name] = dict(ms_per_step=round(ms, 5), value=round(n / (ms * 1e-3), 1),
                         gauge_rel=d["gauge_l2"] / d["gauge_scale"] if d["gauge_scale"] else 0.0,
                         gauss_rel=d["gauss_l2"] / d["gauss_scale"] if d["gauss_scale"] else 0.0)
        ctx.close()
    return out


def bench_variants(steps=40):
    """The current and stepper options on the plain workload (128 x 128,
    64 particles/cell, cubic, float32 particles): v* in J against the plain
    BDF-2 step, the deterministic deposit, and DIRK-2 / DIRK-3 with
    interpolated or sub-stepped stage currents; step rate and the relative
    gauge and Gauss residuals after `steps` steps."""
    import torch
    from paper_2410_18414_amd import pic, workloads
    w = workloads.make("weibel128")
    n = len(w["x"])
    dev = torch.device("cuda:0")
    data = (torch.as_tensor(w["x"], device=dev), torch.as_tensor(w["y"], device=dev),
            torch.as_tensor(np.ascontiguousarray(w["P"].T), device=dev))
    out = dict(workload="weibel-128x128-64ppc-cubic-f32, %d steps" % steps, particles=n, steps=steps)
    variants = (("bdf2", "bdf", 0), ("bdf2_jvstar", "bdf", pic.FLAG_JVSTAR),
                ("bdf2_deterministic", "bdf", pic.FLAG_DETERMINISTIC),
                ("dirk2", "dirk2", 0), ("dirk2_substep", "dirk2", pic.FLAG_DIRK_SUBSTEP),
                ("dirk3", "dirk3", 0), ("dirk3_substep", "dirk3", pic.FLAG_DIRK_SUBSTEP))
    for name, scheme, flags in variants:
        cfg = pic.make_config(w["nx"], w["ny"], w["lx"], w["ly"], w["dt"], degree=3, scheme=scheme, bdf_order=2,
                              dtype="f32", q=w["q"], m=w["m"], max_particles=n, flags=flags)
        ctx = pic.Context(cfg)
        pic.init_particles(ctx, *data)
        pic.step(ctx, pic.graph_period(ctx) + 1)
        pic.init_particles(ctx, *data)
        a, b = _events(ctx.stream)
        torch.cuda.synchronize()
        a.record(ctx.stream)
        pic.step(ctx, steps)
        b.record(ctx.stream)
        torch.cuda.synchronize()
        d = pic.diagnostics(ctx)
        ms = a.elapsed_time(b) / steps
        out[name] = dict(ms_per_step=round(ms, 5), value=round(n / (ms * 1e-3), 1),
                         gauge_rel=d["gauge_l2"] / d["gauge_scale"] if d["gauge_scale"] else 0.0,
                         gauss_rel=d["gauss_l2"] / d["gauss_scale"] if d["gauss_scale"] else 0.0)
        ctx.close()
    return out


def bench_adjoint(every=5):
    """Gradient of the final field energy through 20 BDF-2 steps of the
    128 x 128, 64 particles/cell anisotropic workload with drift (float64,
    cubic, checkpoints every 5 steps) against the plain float64 forward."""
    import torch
    from paper_2410_18414_amd import adjoint, pic, workloads
    w = workloads.make("weibel128-drift")
    nsteps = w["steps"]
    n = len(w["x"])
    dev = torch.device("cuda:0")
    cfg = pic.make_config(w["nx"], w["ny"], w["lx"], w["ly"], w["dt"], degree=3, scheme="bdf", bdf_order=2,
                          dtype="f64", q=w["q"], m=w["m"], max_particles=n, flags=pic.FLAG_ADJOINT)
    ctx = pic.Context(cfg)
    x0 = torch.as_tensor(w["x"], device=dev)
    y0 = torch.as_tensor(w["y"], device=dev)
    P0 = torch.as_tensor(np.ascontiguousarray(w["P"].T), device=dev)
    # plain forward (warm, then timed)
    pic.init_particles(ctx, x0, y0, P0)
    pic.step(ctx, nsteps)
    pic.init_particles(ctx, x0, y0, P0)
    a, b = _events(ctx.stream)
    torch.cuda.synchronize()
    a.record(ctx.stream)
    pic.step(ctx, nsteps)
    b.record(ctx.stream)
    torch.cuda.synchronize()
    ms_fwd = a.elapsed_time(b) / nsteps
    # gradient: checkpointed forward + reverse sweep (warm once, then timed)
    for timed in (False, True):
        xg, yg, Pg = x0.clone().requires_grad_(), y0.clone().requires_grad_(), P0.clone().requires_grad_()
        torch.cuda.synchronize()
        a.record(ctx.stream)
        t0 = time.perf_counter()
        W = adjoint.field_energy(ctx, xg, yg, Pg, nsteps, every=every)
        W.backward()
        b.record(ctx.stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    ms_grad = a.elapsed_time(b)
    ctx.close()
    return dict(workload="weibel-128x128-64ppc-drift0.1-cubic-bdf2-f64, gradient of the field energy after "
                         "%d steps, checkpoints every %d" % (nsteps, every), particles=n, steps=nsteps,
                forward_ms_per_step=round(ms_fwd, 5), gradient_ms=round(ms_grad, 3),
                gradient_wall_s=round(wall, 4),
                gradient_ms_per_step=round(ms_grad / nsteps, 5),
                gradient_vs_forward=round(ms_grad / (ms_fwd * nsteps), 2),
                particle_steps_per_s=round(n * nsteps / (ms_grad * 1e-3), 1))


def kernel_label(spec, nx, ny, tile_cells=0, slack=0):
    """The fused pass's template instance: k_tiled<T, degree, MODE_FUSED = 2,
    tile edge, slack>; the compiled window geometries (16- or 8-cell tiles with
    a slack of 3) run on power-of-two grids, every other plan on <.., 0, 0>."""
    t = "float" if spec["dtype"] == "f32" else "double"
    pow2 = not (nx & (nx - 1) or ny & (ny - 1))
    ts = tile_cells or 16
    while ts > min(nx, ny):
        ts //= 2
    sl = slack or 3
    geo = (ts, sl) if pow2 and sl == 3 and ts in (16, 8) else (0, 0)
    return "k_tiled<%s, %d, 2, %d, %d>" % (t, spec["degree"], geo[0], geo[1])


def measure_plain(w, spec, args, steps, warmup, repeats, flags=0, traffic_tag=None):
    """Throughput of `step` on one workload: `warmup` untimed steps, then
    `repeats` timed regions of exactly `steps` steps each (HIP events on the
    library's stream, bracketed by device synchronisations), reported as the
    median; then one more region of `steps` steps with HIP events around every
    launch group (kernel durations for the roofline)."""
    import torch
    from paper_2410_18414_amd import pic
    n = len(w["x"])
    cfg = pic.make_config(w["nx"], w["ny"], w["lx"], w["ly"], w["dt"], degree=spec["degree"],
                          scheme=spec["scheme"], bdf_order=spec["bdf_order"], dtype=spec["dtype"],
                          q=w["q"], m=w["m"], max_particles=n, flags=flags,
                          sort_interval=args.sort_interval, tile_cells=args.tile_cells,
                          chunk=args.chunk, slack=args.slack)
    ctx = pic.Context(cfg, device="cuda:0")
    dev = ctx.device
    pic.init_particles(ctx, torch.as_tensor(w["x"], device=dev), torch.as_tensor(w["y"], device=dev),
                       torch.as_tensor(np.ascontiguousarray(w["P"].T), device=dev))
    # untimed warm-up; when a timed region is long enough to replay the
    # captured step graph, the warm-up spans one graph period plus a step so
    # that the one-time capture stays out of the timed regions
    period = pic.graph_period(ctx)
    if period and steps - 1 >= period:
        warmup = max(warmup, period + 1)
    pic.step(ctx, warmup)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps, walls = [], []
    for _ in range(repeats):
        torch.cuda.synchronize()
        start.record(ctx.stream)
        t0 = time.perf_counter()
        pic.step(ctx, steps)
        stop.record(ctx.stream)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        reps.append(start.elapsed_time(stop))
    ms = float(np.median(reps))
    # kernel durations: the same number of steps with events around every launch group
    pic.set_kernel_timing(ctx, True)
    pic.kernel_timing(ctx)  # reset
    torch.cuda.synchronize()
    start.record(ctx.stream)
    pic.step(ctx, steps)
    stop.record(ctx.stream)
    torch.cuda.synchronize()
    ms_events = start.elapsed_time(stop)
    kt = pic.kernel_timing(ctx)
    pic.set_kernel_timing(ctx, False)
    diag = pic.diagnostics(ctx)
    ctx.close()
    fused_ms, fused_n = kt["fused"]
    if fused_n == 0:  # unfused run: deposit + gather/push stand in for the fused pass
        fused_ms, fused_n = kt["deposit"][0] + kt["gather_push"][0], max(kt["gather_push"][1], 1)
    avg_fused = fused_ms / max(fused_n, 1)
    alg = n * particle_bytes(spec["dtype"]) + grid_bytes(w["nx"], w["ny"], spec["dtype"])
    achieved = alg / (avg_fused * 1e-3) / 1e9 if avg_fused > 0 else 0.0
    traffic = measured_traffic(traffic_tag) if traffic_tag else None
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                # the rocprofv3-measured bytes over the same live launch time
                traffic_gbs=round(traffic / (avg_fused * 1e-3) / 1e9, 1) if traffic and avg_fused > 0 else None,
                traffic_frac=(round(traffic / (avg_fused * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                              if traffic and avg_fused > 0 else None),
                kernel=kernel_label(spec, w["nx"], w["ny"], args.tile_cells, args.slack)
                + " (fused gather/push/position/deposit)",
                avg_launch_us=round(avg_fused * 1e3, 2), launches=int(fused_n),
                algorithmic_bytes_per_launch=int(alg))
    return dict(n=n, warmup=warmup, ms=ms, reps=reps, wall=walls, ms_events=ms_events, kt=kt,
                roofline=roof, diag=diag)


def workload_config(label, w, spec):
    return {"workload": label, "grid": [w["nx"], w["ny"]], "particles": len(w["x"]),
            "ppc": len(w["x"]) // (w["nx"] * w["ny"]), "spline_degree": spec["degree"],
            "scheme": spec["scheme"] + (str(spec["bdf_order"]) if spec["scheme"] == "bdf" else ""),
            "particle_dtype": spec["dtype"], "field_dtype": "f64"}


def section(label, w, spec, res, steps):
    """A secondary workload's figures (same protocol as the headline)."""
    d = res["diag"]
    return dict(workload=label, particles=res["n"], steps=steps, repeats=len(res["reps"]),
                ms_per_step=round(res["ms"] / steps, 5),
                value=round(res["n"] * steps / (res["ms"] * 1e-3), 1),
                repeat_ms_per_step=[round(r / steps, 5) for r in res["reps"]],
                roofline=res["roofline"],
                kernels_ms_per_step={k: round(v[0] / max(steps, 1), 5) for k, v in res["kt"].items()},
                gauge_rel=d["gauge_l2"] / d["gauge_scale"] if d["gauge_scale"] else 0.0,
                config=workload_config(label, w, spec))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--repeats", type=int, default=5, help="timed regions of --steps steps; the median is reported")
    ap.add_argument("--workload", default="weibel512-dirk2", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-particles", type=int, default=1 << 21,
                    help="particles of the oracle's bounded sample (the first ones of the workload)")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--unfused", action="store_true", help="run deposit and gather/push as separate kernels")
    ap.add_argument("--no-sort", action="store_true", help="plain global-atomic kernels, no tile sort")
    ap.add_argument("--sort-interval", type=int, default=0)
    ap.add_argument("--tile-cells", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--slack", type=int, default=0)
    ap.add_argument("--no-sections", action="store_true",
                    help="skip the second 512x512 stepper and the 128x128 workload")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-instance ensemble section")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint (gradient) section")
    ap.add_argument("--no-naive", action="store_true", help="skip the naive charge-deposit comparison section")
    ap.add_argument("--no-variants", action="store_true", help="skip the current/stepper options section")
    ap.add_argument("--batched-steps", type=int, default=20)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device three times (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2410_18414_amd import workloads

    wid, over, label = WORKLOADS[args.workload]
    w = workloads.make(wid)
    spec = dict(degree=w["degree"], scheme=over.get("scheme", w["scheme"]),
                bdf_order=w["bdf_order"], dtype=w["dtype"])
    n = len(w["x"])
    torch.cuda.set_device(0)
    if args.copy_probe:
        # a plain copy of known size: the FETCH_SIZE / WRITE_SIZE it reads scale
        # the counters of the particle pass to bytes
        src = torch.ones(args.copy_probe << 18, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    from paper_2410_18414_amd import pic
    flags = (pic.FLAG_UNFUSED_STEP if args.unfused else 0) | (pic.FLAG_NO_SORT if args.no_sort else 0)
    default_launch = not (args.unfused or args.no_sort or args.sort_interval or args.tile_cells
                          or args.chunk or args.slack)
    res = measure_plain(w, spec, args, args.steps, args.warmup, args.repeats, flags=flags,
                        traffic_tag=args.workload if default_launch else None)
    ms_step = res["ms"] / args.steps
    value = n * args.steps / (res["ms"] * 1e-3)
    diag = res["diag"]
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": res["warmup"], "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": spec["dtype"], "data": "synthetic",
        "config": dict(workload_config(label, w, spec), parallelism="single-gpu"),
        "roofline": res["roofline"],
        "repeats": args.repeats,
        "repeat_ms_per_step": [round(r / args.steps, 5) for r in res["reps"]],
        "kernels_ms_per_step": {k: round(v[0] / max(args.steps, 1), 5) for k, v in res["kt"].items()},
        "ms_per_step_event_pass": round(res["ms_events"] / args.steps, 5),
        "wall_s": round(float(np.median(res["wall"])), 4),
        "gauge_rel": diag["gauge_l2"] / diag["gauge_scale"] if diag["gauge_scale"] else 0.0,
    }
    if not args.no_sections:
        # the other stepper on the same 512x512 particles, and the 128x128 workload
        others = {"weibel512-dirk2": "weibel512-cdf2", "weibel512-cdf2": "weibel512-dirk2"}
        todo = ([others[args.workload]] if args.workload in others else []) + \
               (["weibel128"] if args.workload != "weibel128" else [])
        for name in todo:
            wid2, over2, label2 = WORKLOADS[name]
            w2 = w if wid2 == wid else workloads.make(wid2)
            spec2 = dict(degree=w2["degree"], scheme=over2.get("scheme", w2["scheme"]),
                         bdf_order=w2["bdf_order"], dtype=w2["dtype"])
            r2 = measure_plain(w2, spec2, args, args.steps, args.warmup, args.repeats, flags=flags,
                               traffic_tag=name if default_launch else None)
            out[name] = section(label2, w2, spec2, r2, args.steps)
    if not args.no_batched:
        out["batched"] = bench_batched(args.batched_steps, 6)
        out["batched_integer_sides"] = bench_batched_integer_sides()
    if not args.no_adjoint:
        out["adjoint"] = bench_adjoint()
        # the same gradient storing every state (no replay)
        store_all = bench_adjoint(every=1)
        out["adjoint"]["store_every_state"] = {k: store_all[k] for k in (
            "gradient_ms", "gradient_vs_forward", "forward_ms_per_step")}
    if not args.no_naive:
        out["naive"] = bench_naive()
    if not args.no_variants:
        out["variants"] = bench_variants()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, spec, args.cpu_particles, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
