"""Sub-stepped DIRK stage currents on the GPU (PIC_FLAG_DIRK_SUBSTEP), against
the oracle's dirk_substep mode (needs an MI355X).

Stage i deposits its current from the particles advanced over c_i dt, and the
stage charge densities are the RK stage values of the continuity equation.
Checked here: the stage currents of one deposit, then particle state and
spectral history through step() (1e-10 float64, 1e-4 float32; tiled and
untiled passes, with v* in J, uneven calls ending in graph replay, a
2-instance ensemble); v_phi + c^2 div A and Gauss's law at round-off on the
GPU; unsupported combinations refused.
"""

import numpy as np
import pytest
import torch

from paper_2410_18414_amd import pic, workloads
from pic_harness import DT_TOL, compare_particles, gpu_parts, hist_to_flat, make_gpu, make_oracle, rel

pytestmark = pytest.mark.gpu
EPS = np.finfo(float).eps
F = pic.FLAG_DIRK_SUBSTEP


def cloud(nx=32, ny=32, ppc=3, seed=81):
    return workloads.cloud(nx=nx, ny=ny, ppc=ppc, seed=seed, drift=0.2, vth=0.05)


@pytest.mark.parametrize("scheme,degree", [("dirk2", 3), ("dirk3", 2)])
def test_stage_currents_match_oracle(gpu_lib, scheme, degree):
    w = cloud()
    o = make_oracle(w, degree, scheme, dirk_substep=True)
    g = make_gpu(w, degree, scheme, "f64", flags=F)
    o.step(3)
    pic.step(g, 3)
    o.deposit()
    pic.deposit_current(g)
    J = pic.get_field(g, pic.FIELD_J).cpu().numpy()
    ns = 3 if scheme == "dirk3" else 2
    assert J.shape == (3 * ns, w["ny"], w["nx"])
    assert rel(J, o.J.reshape(3 * ns, w["ny"], w["nx"])) <= 1e-10
    g.close()


CASES = [
    ("dirk2", 3, "f64", 0),
    ("dirk2", 3, "f32", 0),
    ("dirk3", 2, "f64", 0),
    ("dirk3", 3, "f32", 0),
    ("dirk2", 2, "f64", pic.FLAG_NO_SORT),
    ("dirk3", 4, "f64", pic.FLAG_JVSTAR),
]


@pytest.mark.parametrize("scheme,degree,dtype,flags", CASES)
def test_substep_matches_oracle(gpu_lib, scheme, degree, dtype, flags):
    w = cloud()
    print("case", scheme, degree, dtype, flags, flush=True)
    o = make_oracle(w, degree, scheme, jvstar=bool(flags & pic.FLAG_JVSTAR), dirk_substep=True)
    g = make_gpu(w, degree, scheme, dtype, flags=flags | F)
    for n in (1, 6, 5, 20):      # uneven calls; the last one replays captured graphs
        o.step(n)
        pic.step(g, n)
    tol = DT_TOL[dtype]
    errs, bad = compare_particles(gpu_parts(g), o.part, w["lx"], w["ly"], tol)
    assert not bad, errs
    assert rel(pic.get_history(g).cpu().numpy(), hist_to_flat(o.p, o.hist)) <= tol
    if dtype == "f64":
        d = pic.diagnostics(g)
        assert d["gauge_l2"] <= 1e3 * EPS * d["gauge_scale"], d
        assert d["gauss_l2"] <= 1e3 * EPS * d["gauss_scale"], d
    g.close()


def test_substep_ensemble_matches_oracle(gpu_lib):
    ws = [workloads.maxwellian_cloud(nx, ny, ppc, seed, dx=0.1, sigma=0.15, vth=0.1)
          for nx, ny, ppc, seed in ((32, 32, 6, 121), (64, 16, 4, 122))]
    cfgs = [pic.make_config(w["nx"], w["ny"], w["lx"], w["ly"], w["dt"], degree=3, scheme="dirk3",
                            dtype="f64", q=w["q"], m=w["m"], max_particles=len(w["x"]), flags=F)
            for w in ws]
    b = pic.Context(cfgs)
    for i, w in enumerate(ws):
        pic.select_instance(b, i)
        pic.init_particles(b, torch.as_tensor(w["x"], device=b.device), torch.as_tensor(w["y"], device=b.device),
                           torch.as_tensor(np.ascontiguousarray(w["P"].T), device=b.device))
    pic.step_batched(b, 8)
    for i, w in enumerate(ws):
        o = make_oracle(w, 3, "dirk3", dirk_substep=True)
        o.step(8)
        pic.select_instance(b, i)
        errs, bad = compare_particles(gpu_parts(b), o.part, w["lx"], w["ly"], 1e-10)
        assert not bad, (i, errs)
        assert rel(pic.get_history(b).cpu().numpy(), hist_to_flat(o.p, o.hist)) <= 1e-10


def test_interpolated_and_substepped_runs_differ(gpu_lib):
    w = cloud(seed=82)
    a = make_gpu(w, 3, "dirk2", "f64")
    b = make_gpu(w, 3, "dirk2", "f64", flags=F)
    pic.step(a, 5)
    pic.step(b, 5)
    assert rel(gpu_parts(b)["P"], gpu_parts(a)["P"]) > 1e-8


@pytest.mark.parametrize("scheme,flags", [("bdf", F), ("cdf2", F), ("dirk2", F | pic.FLAG_NAIVE_RHO),
                                          ("dirk2", F | pic.FLAG_ADJOINT)])
def test_substep_refused(gpu_lib, scheme, flags):
    w = cloud()
    with pytest.raises(pic.PicError) as e:
        make_gpu(w, 3, scheme, "f64", flags=flags)
    assert e.value.status == 2     # PIC_ERR_UNSUPPORTED


def test_substep_refused_beyond_lds(gpu_lib):
    """Three stage regions and the work buffers exceed the LDS at ny = 1024:
    creation fails cleanly."""
    w = workloads.cloud(nx=16, ny=1024, ppc=1, seed=83, drift=0.2, vth=0.05)
    with pytest.raises(pic.PicError) as e:
        make_gpu(w, 2, "dirk3", "f64", flags=F)
    assert e.value.status == 2
