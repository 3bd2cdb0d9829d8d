"""pic_diagnostics_all, the entry point for callers that cannot allocate
device memory (needs an MI355X): its kernels keep their reduction partials in
the library's fixed scratch array, so two calls in a row share it.  Each
call's values must equal pic_diagnostics of every instance, also when the
second call covers a smaller input (fewer instances and particles) than the
first; a context beyond the scratch's instance limit is refused."""

import numpy as np
import pytest
import torch

from paper_2410_18414_amd import pic, workloads
from pic_harness import rel

pytestmark = pytest.mark.gpu


def ensemble(sizes, dtype, seed0):
    ws = [workloads.maxwellian_cloud(nx, ny, ppc, seed0 + i, dx=0.1, sigma=0.15, vth=0.1)
          for i, (nx, ny, ppc) in enumerate(sizes)]
    cfgs = [pic.make_config(w["nx"], w["ny"], w["lx"], w["ly"], w["dt"], degree=3, scheme="bdf", bdf_order=2,
                            dtype=dtype, q=w["q"], m=w["m"], max_particles=len(w["x"])) for w in ws]
    c = pic.Context(cfgs if len(cfgs) > 1 else cfgs[0])
    for i, w in enumerate(ws):
        if len(ws) > 1:
            pic.select_instance(c, i)
        pic.init_particles(c, torch.as_tensor(w["x"], device=c.device), torch.as_tensor(w["y"], device=c.device),
                           torch.as_tensor(np.ascontiguousarray(w["P"].T), device=c.device))
    return c


def reference(c):
    rows = []
    for i in range(pic.instance_count(c)):
        if pic.instance_count(c) > 1:
            pic.select_instance(c, i)
        d = pic.diagnostics(c)
        rows.append([d[k] for k in pic.DIAG_NAMES])
    return np.array(rows)


def test_matches_pic_diagnostics_on_consecutive_calls(gpu_lib):
    big = ensemble([(32, 32, 6), (64, 16, 4), (24, 40, 5), (16, 16, 9)], "f64", 300)
    pic.step_batched(big, 7)
    got = pic.diagnostics_all(big).cpu().numpy()
    ref = reference(big)
    assert got.shape == (4, 8)
    for i in range(4):
        assert rel(got[i], ref[i]) <= 1e-12, (i, got[i], ref[i])
    assert np.all(ref[:, 1] > 0) and np.all(ref[:, 5] > 0)  # non-trivial fields
    # second call, a smaller input: one instance, fewer particles (the scratch
    # still holds the first call's partials)
    small = ensemble([(16, 16, 3)], "f32", 310)
    pic.step(small, 4)
    got2 = pic.diagnostics_all(small).cpu().numpy()
    ref2 = reference(small)
    assert got2.shape == (1, 8)
    assert rel(got2[0], ref2[0]) <= 1e-12, (got2[0], ref2[0])
    big.close()
    small.close()


def test_instances_beyond_the_scratch_refused(gpu_lib):
    c = ensemble([(8, 8, 1)] * (pic.DIAG_ALL_MAX + 1), "f32", 400)
    with pytest.raises(pic.PicError):
        pic.diagnostics_all(c)
    c.close()
