"""The deterministic deposit (PIC_FLAG_DETERMINISTIC) on the GPU (needs an
MI355X).

J is summed in 64-bit integers at one fixed scale per instance, so runs repeat
bit for bit whatever order particles and workgroups arrive in.  Checked here:
two runs are identical (float32 and float64; BDF-2, DIRK-2 and sub-stepped
DIRK-3; across sorts and graph replays); the result does not depend on the tile
edge, on fused or unfused steps, or on the sort interval (the window and the
global fallback round every contribution to the same integer); an ensemble
equals its instances run alone, bit for bit; a run resumed from exported state
equals the uninterrupted run, bit for bit; the oracle agrees (1e-10 float64,
1e-4 float32), the J export included.
"""

import numpy as np
import pytest
import torch

from paper_2410_18414_amd import pic, workloads
from pic_harness import DT_TOL, compare_particles, gpu_parts, hist_to_flat, make_gpu, make_oracle, rel

pytestmark = pytest.mark.gpu
DET = pic.FLAG_DETERMINISTIC


def plasma(nx=32, ny=32, ppc=4, seed=131):
    return workloads.weibel(nx=nx, ny=ny, ppc=ppc, seed=seed)


def state(ctx):
    return pic.get_particles(ctx).cpu(), pic.get_history(ctx).cpu()


def same(a, b):
    return all(torch.equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("scheme,dtype,flags", [("bdf", "f32", 0), ("bdf", "f64", 0), ("dirk2", "f32", 0),
                                                ("dirk3", "f64", pic.FLAG_DIRK_SUBSTEP)])
def test_runs_repeat_bit_for_bit(gpu_lib, scheme, dtype, flags):
    w = plasma()
    runs = []
    for _ in range(2):
        g = make_gpu(w, 3, scheme, dtype, flags=flags | DET)
        for n in (1, 30, 7):
            pic.step(g, n)
        runs.append(state(g))
        g.close()
    assert same(runs[0], runs[1])


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_independent_of_tiles_fusion_and_sort_interval(gpu_lib, dtype):
    w = plasma(seed=132)
    ref = None
    for kw in (dict(), dict(tile_cells=8), dict(flags=pic.FLAG_UNFUSED_STEP), dict(sort_interval=1),
               dict(sort_interval=40)):
        flags = kw.pop("flags", 0) | DET
        n = w["x"].shape[0]
        cfg = pic.make_config(w["nx"], w["ny"], w["lx"], w["ly"], w["dt"], degree=3, scheme="bdf", bdf_order=2,
                              dtype=dtype, q=w["q"], m=w["m"], max_particles=n, flags=flags, **kw)
        g = pic.Context(cfg)
        pic.init_particles(g, torch.as_tensor(w["x"], device=g.device), torch.as_tensor(w["y"], device=g.device),
                           torch.as_tensor(np.ascontiguousarray(w["P"].T), device=g.device))
        pic.step(g, 25)
        st = state(g)
        g.close()
        if ref is None:
            ref = st
        else:
            assert same(st, ref), kw


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_fast_particles_leaving_their_windows(gpu_lib, dtype):
    """In-plane speeds near c (proper velocity spread 0.9c, isotropic) move a
    particle a third of a cell per step, so between sorts 40 steps apart most
    particles outrun the 3-cell slack and gather and deposit through the
    global-memory paths; the window and global paths sum in the same order and
    round at the same scale, so the state is still identical bit for bit to
    runs that re-sort every step or use other tiles, and a run resumed at
    another point of the sort cycle equals the uninterrupted one."""
    w = workloads.weibel(nx=32, ny=32, ppc=4, seed=135, vth=0.9, aniso=1.0)
    n = w["x"].shape[0]

    def run(steps, start=None, **kw):
        cfg = pic.make_config(w["nx"], w["ny"], w["lx"], w["ly"], w["dt"], degree=3, scheme="bdf", bdf_order=2,
                              dtype=dtype, q=w["q"], m=w["m"], max_particles=n, flags=DET, **kw)
        g = pic.Context(cfg)
        pic.init_particles(g, torch.as_tensor(w["x"], device=g.device), torch.as_tensor(w["y"], device=g.device),
                           torch.as_tensor(np.ascontiguousarray(w["P"].T), device=g.device))
        if start is not None:
            pic.set_particles(g, start[0].to(g.device))
            pic.set_history(g, start[1].to(g.device))
        pic.step(g, steps)
        st = state(g)
        g.close()
        return st

    ref = run(50, sort_interval=40)
    v = ref[0][5:7].abs().max()
    assert float(v) > 0.5  # in-plane speeds above c/2
    for kw in (dict(sort_interval=1), dict(tile_cells=8, sort_interval=40), dict(sort_interval=7)):
        assert same(run(50, **kw), ref), kw
    mid = run(23, sort_interval=40)
    assert same(run(27, start=mid, sort_interval=40), ref)


def test_matches_oracle_and_atomic_mode(gpu_lib):
    w = plasma(seed=133)
    for dtype in ("f64", "f32"):
        o = make_oracle(w, 3, "bdf", 2)
        g = make_gpu(w, 3, "bdf", dtype, flags=DET)
        a = make_gpu(w, 3, "bdf", dtype)
        o.step(4)
        pic.step(g, 4)
        pic.step(a, 4)
        o.deposit()
        pic.deposit_current(g)
        J = pic.get_field(g, pic.FIELD_J).cpu().numpy()
        assert rel(J, o.J) <= DT_TOL[dtype], (dtype, rel(J, o.J))
        o.solve()
        o.gather_push()
        pic.field_solve(g)
        pic.gather_push(g)
        pic.step(a, 1)
        for n in (6, 5):
            o.step(n)
            pic.step(g, n)
            pic.step(a, n)
        tol = DT_TOL[dtype]
        errs, bad = compare_particles(gpu_parts(g), o.part, w["lx"], w["ly"], tol)
        assert not bad, (dtype, errs)
        assert rel(pic.get_history(g).cpu().numpy(), hist_to_flat(o.p, o.hist)) <= tol
        assert rel(pic.get_history(g).cpu().numpy(), pic.get_history(a).cpu().numpy()) <= tol
        g.close()
        a.close()


def test_ensemble_equals_instances_bit_for_bit(gpu_lib):
    ws = [workloads.maxwellian_cloud(nx, ny, ppc, seed, dx=0.1, sigma=0.15, vth=0.1)
          for nx, ny, ppc, seed in ((32, 32, 6, 141), (64, 16, 4, 142), (24, 40, 5, 143))]
    cfgs = [pic.make_config(w["nx"], w["ny"], w["lx"], w["ly"], w["dt"], degree=3, scheme="bdf", bdf_order=2,
                            dtype="f32", q=w["q"], m=w["m"], max_particles=len(w["x"]), flags=DET) for w in ws]
    b = pic.Context(cfgs)
    for i, w in enumerate(ws):
        pic.select_instance(b, i)
        pic.init_particles(b, torch.as_tensor(w["x"], device=b.device), torch.as_tensor(w["y"], device=b.device),
                           torch.as_tensor(np.ascontiguousarray(w["P"].T), device=b.device))
    pic.step_batched(b, 20)
    for i, w in enumerate(ws):
        a = make_gpu(w, 3, "bdf", "f32", flags=DET)
        pic.step(a, 20)
        pic.select_instance(b, i)
        assert same(state(b), state(a)), i
        a.close()


def test_resume_equals_uninterrupted_bit_for_bit(gpu_lib):
    w = plasma(seed=134)
    full = make_gpu(w, 3, "bdf", "f32", flags=DET)
    pic.step(full, 30)
    first = make_gpu(w, 3, "bdf", "f32", flags=DET)
    pic.step(first, 13)
    parts, hist = pic.get_particles(first), pic.get_history(first)
    first.close()
    resumed = make_gpu(w, 3, "bdf", "f32", flags=DET)
    pic.set_particles(resumed, parts)
    pic.set_history(resumed, hist)
    pic.step(resumed, 17)
    assert same(state(resumed), state(full))
