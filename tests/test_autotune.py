"""Autotuner: plan application (CPU) and a real tuning run (GPU)."""

import json
import os

import pytest

from paper_2410_18414_amd import autotune, pic, workloads


def _cfgs():
    return [pic.make_config(32, 64, 3.2, 6.4, 0.05, degree=3, dtype="f32", max_particles=100),
            pic.make_config(256, 128, 25.6, 12.8, 0.05, degree=3, dtype="f32", max_particles=100,
                            flags=pic.FLAG_NO_GRAPH)]


def test_apply_sets_knobs_and_keeps_the_rest():
    cfgs = _cfgs()
    out = autotune.apply(cfgs, dict(tile_cells=16, chunk=512, unfused=True, sort_interval=9))
    for a, b in zip(cfgs, out):
        assert b.tile_cells == 16 and b.chunk == 512 and b.sort_interval == 9
        assert b.flags & pic.FLAG_UNFUSED_STEP
        assert (b.flags & ~pic.FLAG_UNFUSED_STEP) == a.flags
        assert (b.nx, b.ny, b.lx, b.dt, b.max_particles) == (a.nx, a.ny, a.lx, a.dt, a.max_particles)
    out = autotune.apply(out, dict(tile_cells=64, chunk=1024, unfused=False))
    assert out[0].tile_cells == 32 and not out[0].flags & pic.FLAG_UNFUSED_STEP  # clamped to the grid
    for c in out:
        assert pic.load().pic_workspace_bytes(c) > 0


def test_candidates_are_valid_configs():
    for cand in autotune.CANDIDATES:
        for c in autotune.apply(_cfgs(), cand):
            assert pic.load().pic_workspace_bytes(c) > 0, cand


def test_ensemble_draw_is_seeded_and_in_range():
    a = workloads.ensemble(count=8)
    b = workloads.ensemble(count=8)
    for wa, wb in zip(a, b):
        assert (wa["nx"], wa["ny"]) == (wb["nx"], wb["ny"])
        assert wa["nx"] in (32, 64, 128, 256) and wa["ny"] in (32, 64, 128, 256)
        ppc = len(wa["x"]) // (wa["nx"] * wa["ny"])
        assert 4 <= ppc <= 64 and len(wa["x"]) == ppc * wa["nx"] * wa["ny"]
        assert (wa["x"] == wb["x"]).all()


@pytest.mark.gpu
def test_tune_measures_and_caches(gpu_lib, tmp_path):
    import torch
    ws = [workloads.maxwellian_cloud(32, 32, 8, 7), workloads.maxwellian_cloud(64, 32, 4, 8)]

    def make_cfgs():
        return [pic.make_config(w["nx"], w["ny"], w["lx"], w["ly"], w["dt"], degree=3, dtype="f32", q=w["q"],
                                m=w["m"], max_particles=len(w["x"])) for w in ws]

    def load(ctx):
        for i, w in enumerate(ws):
            pic.select_instance(ctx, i)
            pic.init_particles(ctx, torch.as_tensor(w["x"], device="cuda"), torch.as_tensor(w["y"], device="cuda"),
                               torch.as_tensor(w["P"].T.copy(), device="cuda"))

    path = str(tmp_path / "tune.json")
    cands = autotune.CANDIDATES[:3]
    plan = autotune.tune("two-clouds", make_cfgs, load, candidates=cands, steps=3, warmup=2, cache_path=path)
    assert not plan["cached"] and len(plan["results"]) == 3
    assert all(r["ms_per_step"] > 0 for r in plan["results"])
    again = autotune.tune("two-clouds", make_cfgs, load, candidates=cands, cache_path=path)
    assert again["cached"] and {k: again[k] for k in autotune.KNOBS} == {k: plan[k] for k in autotune.KNOBS}
    assert len(json.load(open(path))) == 1
