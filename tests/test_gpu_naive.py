"""The naive charge-deposit comparison on the GPU (PIC_FLAG_NAIVE_RHO), against
the oracle's naive mode (needs an MI355X).

The naive update of the Weibel figures (Sec. 5.1) maps rho^{n+1} to the mesh
with the same spline as J instead of updating it from continuity.  Checked
here: particle state and spectral history equal the oracle's naive run
(1e-10 float64, 1e-4 float32) on the tiled passes (with a fourth LDS window
plane for rho) and on the untiled ones; the gauge and Gauss residuals equal the
oracle's (both far above round-off, while the continuity run keeps the gauge
at round-off); particles at rest keep rho = 0; unsupported combinations are
rejected before anything runs.
"""

import numpy as np
import pytest
import torch

from oracle import diagnostics as odiag
from paper_2410_18414_amd import pic, workloads
from pic_harness import DT_TOL, compare_particles, gpu_parts, hist_to_flat, make_gpu, make_oracle, rel

pytestmark = pytest.mark.gpu
EPS = np.finfo(float).eps


def cloud(nx=32, ny=32, ppc=3, seed=31):
    return workloads.cloud(nx=nx, ny=ny, ppc=ppc, seed=seed, drift=0.2, vth=0.05)


@pytest.mark.parametrize("scheme,k,degree", [("bdf", 1, 2), ("bdf", 2, 3), ("dirk2", 2, 2)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("extra", [0, pic.FLAG_NO_SORT], ids=["tiled", "untiled"])
def test_naive_matches_oracle(gpu_lib, scheme, k, degree, dtype, extra):
    w = cloud()
    o = make_oracle(w, degree, scheme, k, naive=True)
    g = make_gpu(w, degree, scheme, dtype, bdf_order=k, flags=pic.FLAG_NAIVE_RHO | extra)
    for n in (1, 6, 5):          # uneven call lengths (direct launches and graph-free steps)
        o.step(n)
        pic.step(g, n)
    tol = DT_TOL[dtype]
    errs, bad = compare_particles(gpu_parts(g), o.part, w["lx"], w["ly"], tol)
    assert not bad, errs
    assert rel(pic.get_history(g).cpu().numpy(), hist_to_flat(o.p, o.hist)) <= tol
    if dtype == "f64":
        dg, do = pic.diagnostics(g), odiag.residuals(o)
        assert rel(dg["gauge_l2"], do["gauge_l2"]) <= 1e-8
        assert rel(dg["gauss_l2"], do["gauss_l2"]) <= 1e-8
        assert dg["gauge_l2"] >= 1e-6 * dg["gauge_scale"]     # the naive update breaks the gauge
    g.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_naive_charge_of_particles_leaving_their_windows(gpu_lib, dtype):
    """Fast particles and a long sort interval: stencils that leave their
    tile's window deposit rho (and J) with global atomics.  The run equals the
    one that re-sorts every step (every stencil in its window) to the
    precision's tolerance."""
    w = workloads.cloud(nx=32, ny=32, ppc=4, seed=34, drift=0.3, vth=0.6)
    runs = []
    for si in (40, 1):
        g = make_gpu(w, 3, "bdf", dtype, bdf_order=2, flags=pic.FLAG_NAIVE_RHO, sort_interval=si)
        pic.step(g, 24)
        runs.append((gpu_parts(g), pic.get_history(g).cpu().numpy()))
        g.close()
    tol = DT_TOL[dtype]
    assert rel(runs[0][1], runs[1][1]) <= tol
    errs, bad = compare_particles(runs[0][0], runs[1][0], w["lx"], w["ly"], tol)
    assert not bad, errs


def test_continuity_keeps_gauge_naive_breaks_it(gpu_lib):
    w = cloud(seed=32)
    cons = make_gpu(w, 2, "bdf", "f64")
    naive = make_gpu(w, 2, "bdf", "f64", flags=pic.FLAG_NAIVE_RHO)
    pic.step(cons, 20)
    pic.step(naive, 20)
    dc, dn = pic.diagnostics(cons), pic.diagnostics(naive)
    assert dc["gauge_l2"] <= 1e3 * EPS * dc["gauge_scale"], dc
    assert dc["gauss_l2"] <= 1e3 * EPS * dc["gauss_scale"], dc
    assert dn["gauge_l2"] >= 1e-6 * dn["gauge_scale"], dn
    assert dn["gauss_l2"] >= 1e-6 * dn["gauss_scale"], dn


@pytest.mark.parametrize("scheme", ["bdf", "dirk2"])
def test_naive_particles_at_rest_keep_zero_charge(gpu_lib, scheme):
    w = cloud(seed=33)
    w = dict(w, P=0.0 * w["P"])
    g = make_gpu(w, 3, scheme, "f64", flags=pic.FLAG_NAIVE_RHO)
    pic.step(g, 4)
    H = pic.get_history(g).cpu().numpy()
    # rho levels first in the export order: round-off of bg + deposit only
    scale = abs(w["q"]) * len(w["x"]) / (w["lx"] * w["ly"])
    assert np.abs(H).max() <= 1e-12 * scale * w["nx"] * w["ny"]
    g.close()


@pytest.mark.parametrize("flags,scheme", [(pic.FLAG_NAIVE_RHO, "cdf2"),
                                          (pic.FLAG_NAIVE_RHO | pic.FLAG_ADJOINT, "bdf")])
def test_naive_rejects_unsupported(gpu_lib, flags, scheme):
    w = cloud()
    with pytest.raises(pic.PicError) as e:
        make_gpu(w, 2, scheme, "f64", flags=flags)
    assert e.value.status == 2     # PIC_ERR_UNSUPPORTED
