"""Checkpoint files, device-resident saved states (pic_save_state /
pic_load_state, and the _h forms that keep the header on the host) and the
diagnostics log on the GPU (needs an MI355X): a deterministic run resumed from
a checkpoint file or from a saved state equals the uninterrupted run bit for
bit (in the same context, in a fresh one, in an ensemble, with the naive charge
deposit, with the header taken from the host); both refuse a context of another
configuration and a header of another one; the log has one line per interval with the gauge residual at
round-off."""

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


def _same(a, b, tol=0.0):
    pa, pb = pic.get_particles(a).cpu(), pic.get_particles(b).cpu()
    ha, hb = pic.get_history(a).cpu(), pic.get_history(b).cpu()
    if tol == 0.0:
        assert torch.equal(pa, pb) and torch.equal(ha, hb)
    else:
        assert float((pa - pb).abs().max() / pb.abs().max()) <= tol
        assert float((ha - hb).abs().max() / hb.abs().max()) <= tol


# the deterministic deposit repeats runs bit for bit; the naive charge deposit
# is not available with it, so that case compares within the float64 atomic
# summation order (1e-10 after 18 steps, as for ensembles)
@pytest.mark.parametrize("dtype,scheme,k,flags,tol", [
    ("f32", "bdf", 3, pic.FLAG_DETERMINISTIC, 0.0), ("f64", "bdf", 2, pic.FLAG_DETERMINISTIC, 0.0),
    ("f32", "dirk2", 2, pic.FLAG_DETERMINISTIC, 0.0), ("f64", "dirk3", 2, pic.FLAG_DETERMINISTIC, 0.0),
    ("f32", "cdf2", 2, pic.FLAG_DETERMINISTIC, 0.0),
    ("f32", "dirk2", 2, pic.FLAG_DETERMINISTIC | pic.FLAG_DIRK_SUBSTEP, 0.0),
    ("f64", "bdf", 2, pic.FLAG_NAIVE_RHO, 1e-10)])
def test_saved_state_resume(gpu_lib, dtype, scheme, k, flags, tol):
    w = workloads.weibel(nx=32, ny=24, ppc=4, seed=153)
    full = make_gpu(w, 3, scheme, dtype, bdf_order=k, flags=flags)
    pic.step(full, 31)
    a = make_gpu(w, 3, scheme, dtype, bdf_order=k, flags=flags)
    pic.step(a, 13)
    saved = pic.save_state(a)
    pic.step(a, 18)                       # saving leaves the run undisturbed
    _same(a, full, tol)
    pic.load_state(a, saved)              # back to step 13 in the same context
    pic.step(a, 18)
    _same(a, full, tol)
    b = make_gpu(w, 3, scheme, dtype, bdf_order=k, flags=flags)
    pic.load_state(b, saved)              # into another context of the configuration
    pic.step(b, 7)
    pic.step(b, 11)
    _same(b, full, tol)
    pic.load_state(b, saved, trust_header=True)   # the header from the host: no read of the buffer
    pic.step(b, 18)
    _same(b, full, tol)
    d_full, d_b = pic.diagnostics(full), pic.diagnostics(b)
    for key in ("energy", "kinetic"):
        assert abs(d_b[key] - d_full[key]) <= max(tol, 1e-12) * abs(d_full[key]), key


def test_saved_state_ensemble_and_refusals(gpu_lib):
    ws = [workloads.maxwellian_cloud(nx, ny, ppc, seed, dx=0.1, sigma=0.15, vth=0.1)
          for nx, ny, ppc, seed in [(32, 32, 6, 161), (16, 64, 3, 162), (48, 40, 2, 163)]]

    def ens():
        cfgs = [pic.make_config(w["nx"], w["ny"], w["lx"], w["ly"], w["dt"], scheme="dirk2", dtype="f32",
                                q=w["q"], m=w["m"], max_particles=len(w["x"]) + 17,
                                flags=pic.FLAG_DETERMINISTIC) for w in ws]
        ctx = pic.Context(cfgs)
        for i, w in enumerate(ws):
            pic.select_instance(ctx, i)
            dev = ctx.device
            pic.init_particles(ctx, torch.as_tensor(w["x"], device=dev), torch.as_tensor(w["y"], device=dev),
                               torch.as_tensor(np.ascontiguousarray(w["P"].T), device=dev))
        return ctx

    full = ens()
    pic.step_batched(full, 20)
    a = ens()
    pic.step_batched(a, 9)
    saved = pic.save_state(a)
    b = pic.Context(a.cfgs)               # never loaded: phase EMPTY
    pic.load_state(b, saved)
    pic.step_batched(b, 11)
    for i in range(len(ws)):
        pic.select_instance(full, i)
        pic.select_instance(b, i)
        assert b.n == full.n == len(ws[i]["x"])
        _same(b, full)
    # another configuration, a misaligned buffer and a mid-step phase are refused
    c = make_gpu(ws[0], 3, "dirk2", "f32", flags=pic.FLAG_DETERMINISTIC)
    with pytest.raises(pic.PicError):
        pic.load_state(c, saved)
    with pytest.raises(pic.PicError):
        pic.load_state(c, pic.save_state(c))
        pic.deposit_current(c)
        pic.save_state(c)
    # a host header of another configuration is refused (its length, then its words)
    foreign = pic.save_state(make_gpu(ws[0], 3, "dirk2", "f32", flags=pic.FLAG_DETERMINISTIC))
    with pytest.raises(ValueError):
        pic.load_state(b, foreign, trust_header=True)
    other = make_gpu(ws[1], 3, "dirk2", "f32", flags=pic.FLAG_DETERMINISTIC)
    with pytest.raises(pic.PicError):
        pic.load_state(other, foreign, trust_header=True)
    bad = pic.State(a)
    bad.ptr = type(bad.ptr)(bad.ptr.value + 8)
    with pytest.raises(pic.PicError):
        pic.save_state(a, bad)
