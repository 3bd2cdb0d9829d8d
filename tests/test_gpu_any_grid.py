"""Grid sides that are not powers of two (any side in [8, 1024]) on the GPU,
against the oracle (needs an MI355X).

The field solve uses the mixed-radix LDS FFT (radix 4 and 2, then one pass per
odd prime factor); the cell-sorted tiles end in partial tiles at the high
edges and the generic tiled kernel wraps node indices by remainders.  Checked
here:
particle state and spectral history through step() for even, odd and prime
sides, both precisions and the three stepper families (1e-10 float64, 1e-4
float32); uniform plasmas filling partial tiles and crossing the seams,
tiled against untiled; the largest sides (a prime near 1024 along x, 1000 along y); the
gauge residual at round-off; an ensemble whose sides are uniform integers in
[32, 256] (the strict reading of the uneven ensemble); the adjoint refused.
"""

import numpy as np
import pytest
import torch

from paper_2410_18414_amd import pic, workloads
from pic_harness import DT_TOL, compare_particles, gpu_parts, hist_to_flat, make_gpu, make_oracle, rel

pytestmark = pytest.mark.gpu
EPS = np.finfo(float).eps


def cloud(nx, ny, ppc=3, seed=91):
    return workloads.cloud(nx=nx, ny=ny, ppc=ppc, seed=seed, drift=0.2, vth=0.05)


CASES = [
    (24, 20, "bdf", 2, 3, "f64"),
    (27, 15, "bdf", 2, 3, "f32"),
    (37, 29, "cdf2", 2, 2, "f64"),
    (100, 36, "dirk2", 2, 3, "f64"),
    (9, 8, "bdf", 1, 2, "f64"),
    (45, 49, "dirk3", 2, 3, "f32"),
]


@pytest.mark.parametrize("nx,ny,scheme,k,degree,dtype", CASES)
def test_other_grid_matches_oracle(gpu_lib, nx, ny, scheme, k, degree, dtype):
    print("case", nx, ny, scheme, k, degree, dtype, flush=True)
    w = cloud(nx, ny)
    o = make_oracle(w, degree, scheme, k)
    g = make_gpu(w, degree, scheme, dtype, bdf_order=k)
    for n in (1, 4, 7):
        o.step(n)
        pic.step(g, n)
    tol = DT_TOL[dtype]
    errs, bad = compare_particles(gpu_parts(g), o.part, w["lx"], w["ly"], tol)
    assert not bad, errs
    assert rel(pic.get_history(g).cpu().numpy(), hist_to_flat(o.p, o.hist)) <= tol
    if dtype == "f64":
        d = pic.diagnostics(g)
        assert d["gauge_l2"] <= 1e3 * EPS * d["gauge_scale"], d
    g.close()


@pytest.mark.parametrize("nx,ny,dtype", [(36, 20, "f64"), (50, 27, "f32"), (9, 13, "f64")])
def test_uniform_plasma_partial_tiles(gpu_lib, nx, ny, dtype):
    """Uniform positions fill the partial tiles at the high edges and cross
    the periodic seams; tiled (sorted) and untiled runs agree with the oracle
    and, in float64, with each other."""
    print("case", nx, ny, dtype, flush=True)
    w = workloads.weibel(nx=nx, ny=ny, ppc=4, seed=95)
    o = make_oracle(w, 3, "bdf", 2)
    g = make_gpu(w, 3, "bdf", dtype)
    u = make_gpu(w, 3, "bdf", dtype, flags=pic.FLAG_NO_SORT)
    for n in (2, 9, 9):          # several sorts (worst-case interval: slack / (c dt / dx) = 6 steps)
        o.step(n)
        pic.step(g, n)
        pic.step(u, n)
    tol = DT_TOL[dtype]
    for ctx in (g, u):
        errs, bad = compare_particles(gpu_parts(ctx), o.part, w["lx"], w["ly"], tol)
        assert not bad, errs
        assert rel(pic.get_history(ctx).cpu().numpy(), hist_to_flat(o.p, o.hist)) <= tol
    if dtype == "f64":
        assert rel(pic.get_history(g).cpu().numpy(), pic.get_history(u).cpu().numpy()) <= 1e-12
    g.close()
    u.close()


@pytest.mark.parametrize("nx,ny,scheme,flags", [(1021, 10, "bdf", 0), (12, 1000, "bdf", 0),
                                                (16, 1024, "dirk2", 0), (10, 1000, "dirk3", 0),
                                                (16, 1024, "dirk2", pic.FLAG_NAIVE_RHO)])
def test_largest_sides_match_oracle(gpu_lib, nx, ny, scheme, flags):
    """The largest FFT lengths, and DIRK with ny above 512 (its column kernel
    then transforms the J columns one at a time)."""
    print("case", nx, ny, scheme, flags, flush=True)
    w = cloud(nx, ny, ppc=1, seed=92)
    o = make_oracle(w, 2, scheme, 2, naive=bool(flags & pic.FLAG_NAIVE_RHO))
    g = make_gpu(w, 2, scheme, "f64", flags=flags)
    o.step(3)
    pic.step(g, 3)
    errs, bad = compare_particles(gpu_parts(g), o.part, w["lx"], w["ly"], 1e-10)
    assert not bad, errs
    assert rel(pic.get_history(g).cpu().numpy(), hist_to_flat(o.p, o.hist)) <= 1e-10
    g.close()


def test_mesh_fields_match_oracle_on_odd_grid(gpu_lib):
    w = cloud(33, 21, seed=93)
    o = make_oracle(w, 3, "bdf", 2)
    g = make_gpu(w, 3, "bdf", "f64")
    o.step(2)
    pic.step(g, 2)
    o.deposit()
    o.solve()
    pic.deposit_current(g)
    pic.field_solve(g)
    F = pic.get_field(g, pic.FIELD_MESH).cpu().numpy()
    assert rel(F, o.fields) <= 1e-10
    g.close()


def test_ensemble_with_integer_sides_matches_oracle(gpu_lib):
    ws = workloads.ensemble(count=4, sizes=slice(32, 256), ppc_range=(1, 2))
    assert any(w["nx"] & (w["nx"] - 1) for w in ws)     # at least one side is not a power of two
    cfgs = [pic.make_config(w["nx"], w["ny"], w["lx"], w["ly"], w["dt"], degree=3, scheme="bdf", bdf_order=2,
                            dtype="f64", q=w["q"], m=w["m"], max_particles=len(w["x"]))
            for w in ws]
    b = pic.Context(cfgs)
    for i, w in enumerate(ws):
        pic.select_instance(b, i)
        pic.init_particles(b, torch.as_tensor(w["x"], device=b.device), torch.as_tensor(w["y"], device=b.device),
                           torch.as_tensor(np.ascontiguousarray(w["P"].T), device=b.device))
    pic.step_batched(b, 4)
    for i, w in enumerate(ws):
        o = make_oracle(w, 3, "bdf", 2)
        o.step(4)
        pic.select_instance(b, i)
        errs, bad = compare_particles(gpu_parts(b), o.part, w["lx"], w["ly"], 1e-10)
        assert not bad, (i, w["nx"], w["ny"], errs)
        assert rel(pic.get_history(b).cpu().numpy(), hist_to_flat(o.p, o.hist)) <= 1e-10


def test_adjoint_refused_on_other_grids(gpu_lib):
    w = cloud(24, 16)
    with pytest.raises(pic.PicError) as e:
        make_gpu(w, 3, "bdf", "f64", flags=pic.FLAG_ADJOINT)
    assert e.value.status == 2
