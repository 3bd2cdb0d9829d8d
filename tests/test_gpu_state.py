"""Checkpoint files and the diagnostics log (paper_2410_18414_amd.state) on the
GPU (needs an MI355X): a deterministic run resumed from a checkpoint file
equals the uninterrupted run bit for bit; a checkpoint refuses a context of
another configuration; the log has one line per interval with the gauge
residual at round-off."""

import json

import numpy as np
import pytest
import torch

from paper_2410_18414_amd import pic, state, workloads
from pic_harness import make_gpu

pytestmark = pytest.mark.gpu
EPS = np.finfo(float).eps


def test_checkpoint_resume_bit_for_bit(gpu_lib, tmp_path):
    w = workloads.weibel(nx=32, ny=24, ppc=4, seed=151)
    full = make_gpu(w, 3, "bdf", "f32", flags=pic.FLAG_DETERMINISTIC)
    pic.step(full, 30)
    a = make_gpu(w, 3, "bdf", "f32", flags=pic.FLAG_DETERMINISTIC)
    pic.step(a, 12)
    path = str(tmp_path / "ck.npz")
    state.save_state(a, path)
    a.close()
    b = make_gpu(w, 3, "bdf", "f32", flags=pic.FLAG_DETERMINISTIC)
    state.load_state(b, path)
    pic.step(b, 18)
    assert torch.equal(pic.get_particles(b).cpu(), pic.get_particles(full).cpu())
    assert torch.equal(pic.get_history(b).cpu(), pic.get_history(full).cpu())
    # another configuration is refused
    c = make_gpu(w, 2, "bdf", "f32", flags=pic.FLAG_DETERMINISTIC)
    with pytest.raises(ValueError):
        state.load_state(c, path)


def test_diagnostics_log(gpu_lib, tmp_path):
    w = workloads.cloud(nx=32, ny=32, ppc=3, seed=152, drift=0.2, vth=0.05)
    g = make_gpu(w, 2, "bdf", "f64")
    path = str(tmp_path / "diag.jsonl")
    assert state.run_logged(g, 25, 10, path) == 25
    recs = [json.loads(line) for line in open(path)]
    assert [r["step"] for r in recs] == [10, 20, 25]
    for r in recs:
        assert r["gauge_rel"] <= 1e3 * EPS and r["nonfinite"] == 0
        assert np.isfinite(r["energy"]) and np.isfinite(r["kinetic"])
