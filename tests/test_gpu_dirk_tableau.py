"""General s-stage DIRK on the GPU (pic_set_dirk_tableau; needs an MI355X).

Alexander's L-stable two- and three-stage tableaux (not compositions of
implicit-midpoint steps) replace the DIRK-2 / DIRK-3 tableaux: trajectories
and the spectral history through step() match the oracle run with the same
tableau (1e-10 float64, 1e-4 float32), with interpolated and with
sub-stepped stage currents and in an ensemble; the gauge residual stays at
round-off; invalid tableaux and non-DIRK contexts are refused.
"""

import numpy as np
import pytest
import torch

from paper_2410_18414_amd import pic, workloads
from pic_harness import DT_TOL, compare_particles, gpu_parts, hist_to_flat, make_gpu, rel
from oracle import pic as opic
from test_oracle_fields import sdirk

pytestmark = pytest.mark.gpu
EPS = np.finfo(float).eps


def cloud():
    return workloads.cloud(nx=32, ny=32, ppc=3, seed=91, drift=0.2, vth=0.05)


@pytest.mark.parametrize("s", [2, 3])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("substep", [False, True])
def test_trajectory_against_oracle(gpu_lib, s, dtype, substep):
    w = cloud()
    scheme = "dirk2" if s == 2 else "dirk3"
    tab = sdirk(s)
    p = opic.Params(w["nx"], w["ny"], w["lx"], w["ly"], 3, scheme, w["dt"], q=w["q"], m=w["m"],
                    dirk_substep=substep, dirk_tableau=tab)
    o = opic.State(p, w["x"], w["y"], w["P"])
    g = make_gpu(w, 3, scheme, dtype, flags=pic.FLAG_DIRK_SUBSTEP if substep else 0)
    pic.set_dirk_tableau(g, *tab)
    for chunk in (7, 13):  # the second call replays the captured step graph
        o.step(chunk)
        pic.step(g, chunk)
    errs, bad = compare_particles(gpu_parts(g), o.part, w["lx"], w["ly"], DT_TOL[dtype])
    assert not bad, errs
    assert rel(pic.get_history(g).cpu().numpy(), hist_to_flat(p, o.hist)) <= DT_TOL[dtype]
    d = pic.diagnostics(g)
    assert d["gauge_l2"] <= 1e3 * EPS * d["gauge_scale"], d
    g.close()


def test_tableau_changes_the_run_and_applies_to_every_instance(gpu_lib):
    ws = [workloads.maxwellian_cloud(nx, ny, ppc, seed, dx=0.1, sigma=0.15, vth=0.1)
          for nx, ny, ppc, seed in ((32, 32, 4, 92), (24, 40, 3, 93))]
    cfgs = [pic.make_config(w["nx"], w["ny"], w["lx"], w["ly"], w["dt"], degree=3, scheme="dirk2", dtype="f64",
                            q=w["q"], m=w["m"], max_particles=len(w["x"])) for w in ws]
    b = pic.Context(cfgs)
    for i, w in enumerate(ws):
        pic.select_instance(b, i)
        pic.init_particles(b, torch.as_tensor(w["x"], device=b.device), torch.as_tensor(w["y"], device=b.device),
                           torch.as_tensor(np.ascontiguousarray(w["P"].T), device=b.device))
    tab = sdirk(2)
    pic.set_dirk_tableau(b, *tab)
    pic.step_batched(b, 10)
    for i, w in enumerate(ws):
        p = opic.Params(w["nx"], w["ny"], w["lx"], w["ly"], 3, "dirk2", w["dt"], q=w["q"], m=w["m"],
                        dirk_tableau=tab)
        o = opic.State(p, w["x"], w["y"], w["P"])
        o.step(10)
        pic.select_instance(b, i)
        errs, bad = compare_particles(gpu_parts(b), o.part, w["lx"], w["ly"], 1e-10)
        assert not bad, (i, errs)
        # the default tableau gives another run
        q = make_gpu(w, 3, "dirk2", "f64")
        pic.step(q, 10)
        assert rel(pic.get_history(q).cpu().numpy(), pic.get_history(b).cpu().numpy()) > 1e-6
        q.close()
    b.close()


def test_invalid_tableaux_refused(gpu_lib):
    w = cloud()
    g = make_gpu(w, 3, "dirk2", "f64")
    A, b, c = sdirk(2)
    bad = [(np.array([[0.3, 0.1], [0.4, 0.3]]), b, c),       # not lower triangular
           (A, b, c + 0.1),                                     # c differs from the row sums
           (A, b * 1.1, c),                                     # weights do not sum to one
           (np.array([[0.0, 0.0], [0.5, 0.5]]), b, np.array([0.0, 1.0]))]  # zero diagonal
    for t in bad:
        with pytest.raises(pic.PicError):
            pic.set_dirk_tableau(g, *t)
    with pytest.raises(pic.PicError):
        pic.set_dirk_tableau(g, *sdirk(3))                     # three stages on DIRK-2
    pic.step(g, 2)
    pic.deposit_current(g)
    with pytest.raises(pic.PicError):
        pic.set_dirk_tableau(g, A, b, c)                       # mid-step
    g.close()
    h = make_gpu(w, 3, "bdf", "f64")
    with pytest.raises(pic.PicError):
        pic.set_dirk_tableau(h, A, b, c)
    h.close()
