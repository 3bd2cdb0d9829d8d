"""Ensemble (batched) contexts: every instance of one context matches the same
instance run alone, on uneven grids and particle counts (needs an MI355X).

float64 at 1e-10 (the instances' deposits differ only in the order of float64
atomic additions), float32 at 1e-5.
"""

import numpy as np
import pytest
import torch

from paper_2410_18414_amd import pic, workloads
from pic_harness import compare_particles, gpu_parts, hist_to_flat, make_gpu, make_oracle, rel

pytestmark = pytest.mark.gpu

SHAPES = [(32, 32, 6, 101), (64, 32, 4, 102), (16, 64, 9, 103), (128, 128, 3, 104), (8, 8, 5, 105),
          (32, 16, 1, 106)]


def members(dtype):
    ws = [workloads.maxwellian_cloud(nx, ny, ppc, seed, dx=0.1, sigma=0.15, vth=0.1)
          for nx, ny, ppc, seed in SHAPES]
    return ws


def batch_ctx(ws, dtype, scheme="bdf", k=2, degree=3):
    cfgs = [pic.make_config(w["nx"], w["ny"], w["lx"], w["ly"], w["dt"], degree=degree, scheme=scheme,
                            bdf_order=k, dtype=dtype, q=w["q"], m=w["m"], max_particles=len(w["x"]))
            for w in ws]
    ctx = pic.Context(cfgs)
    for i, w in enumerate(ws):
        pic.select_instance(ctx, i)
        dev = ctx.device
        pic.init_particles(ctx, torch.as_tensor(w["x"], device=dev), torch.as_tensor(w["y"], device=dev),
                           torch.as_tensor(np.ascontiguousarray(w["P"].T), device=dev))
    return ctx


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 1e-5)])
@pytest.mark.parametrize("scheme,k", [("bdf", 2), ("dirk2", 2)])
def test_batched_equals_plain(gpu_lib, dtype, tol, scheme, k):
    ws = members(dtype)
    b = batch_ctx(ws, dtype, scheme, k)
    assert pic.instance_count(b) == len(ws)
    pic.step_batched(b, 12)
    for i, w in enumerate(ws):
        a = make_gpu(w, 3, scheme, dtype, bdf_order=k)
        pic.step(a, 12)
        pic.select_instance(b, i)
        pa, pb = gpu_parts(a), gpu_parts(b)
        for key in pa:
            assert rel(pb[key], pa[key]) <= tol, (i, key, rel(pb[key], pa[key]))
        ha = pic.get_history(a).cpu().numpy()
        hb = pic.get_history(b).cpu().numpy()
        assert rel(hb, ha) <= tol, (i, rel(hb, ha))


def test_batched_matches_oracle_f64(gpu_lib):
    ws = members("f64")[:4]
    b = batch_ctx(ws, "f64")
    pic.step_batched(b, 6)
    for i, w in enumerate(ws):
        o = make_oracle(w, 3, "bdf", 2)
        o.step(6)
        pic.select_instance(b, i)
        errs, bad = compare_particles(gpu_parts(b), o.part, w["lx"], w["ly"], 1e-10)
        assert not bad, (i, errs)
        assert rel(pic.get_history(b).cpu().numpy(), hist_to_flat(o.p, o.hist)) <= 1e-10
        d = pic.diagnostics(b)
        assert d["gauge_l2"] <= 1e-12 * d["gauge_scale"]


def test_batched_rules(gpu_lib):
    ws = members("f32")[:2]
    b = batch_ctx(ws, "f32")
    pic.step_batched(b, 2)
    pic.select_instance(b, 1)
    w = ws[1]
    with pytest.raises(pic.PicError) as e:       # loading after stepping is refused
        pic.init_particles(b, torch.as_tensor(w["x"], device=b.device),
                           torch.as_tensor(w["y"], device=b.device),
                           torch.as_tensor(np.ascontiguousarray(w["P"].T), device=b.device))
    assert e.value.status == 5
    with pytest.raises(pic.PicError):
        pic.select_instance(b, 2)
