"""GPU-vs-oracle parity through the C ABI (needs an MI355X).

Tolerances (normwise, ||gpu - oracle||_inf / ||oracle||_inf per array):
1e-10 for float64 particle state and 1e-4 for float32 particle state; mesh
fields and spectra are float64 in both cases and get the same bar as the
particle dtype that produced their source J.

Sizes span several FFT tiles and thread blocks with ragged particle counts
(not multiples of the 256-thread block).
"""

import numpy as np
import pytest
import torch

from oracle import diagnostics as odiag
from paper_2410_18414_amd import pic, workloads
from pic_harness import (DT_TOL, compare_particles, gpu_parts, hist_to_flat, make_gpu,
                         make_oracle, rel, set_gpu_parts)

pytestmark = pytest.mark.gpu
EPS = np.finfo(float).eps


def weibel_small(nx=32, ny=16, ppc=7, seed=11, drift=0.1):
    return workloads.weibel(nx=nx, ny=ny, ppc=ppc, seed=seed, drift=drift)


def cloud_small(nx=32, ny=32, ppc=3, seed=12):
    return workloads.cloud(nx=nx, ny=ny, ppc=ppc, seed=seed, drift=0.2, vth=0.05)


# BDF-4..6 are A(alpha)-stable only (Sec. 3.2): on the wave equation's
# imaginary eigenvalues a few modes grow slowly, identically on both sides
# (a 1e-15 perturbation of the cloud run's momenta stays below 2e-14 after
# 30 BDF-6 steps on the oracle)
SCHEMES = [("bdf", 1), ("bdf", 2), ("bdf", 3), ("bdf", 4), ("bdf", 5), ("bdf", 6), ("cdf2", 2), ("dirk2", 2)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("degree", [1, 2, 3, 4, 5])
def test_deposit_parity(gpu_lib, dtype, degree):
    w = weibel_small()
    o = make_oracle(w, degree, "bdf")
    ctx = make_gpu(w, degree, "bdf", dtype)
    Jo = o.deposit()
    pic.deposit_current(ctx)
    Jg = pic.get_field(ctx, pic.FIELD_J).cpu().numpy()
    assert rel(Jg, Jo) <= DT_TOL[dtype]
    gp = gpu_parts(ctx)
    errs, bad = compare_particles(gp, o.part, w["lx"], w["ly"], DT_TOL[dtype])
    assert not bad, errs
    # k = 0 mode: total current equals sum of q v exactly up to rounding
    tot = Jg.sum((1, 2)) * (w["lx"] / w["nx"]) * (w["ly"] / w["ny"])
    # bound by the rounding of the summands, sum |q v|, not of the cancelling total
    scale = np.abs(w["q"] * gp["v"]).sum(0)
    np.testing.assert_allclose(tot, w["q"] * gp["v"].sum(0), rtol=0,
                               atol=(1e-6 if dtype == "f32" else 1e-13) * scale.max())


@pytest.mark.parametrize("scheme,k", SCHEMES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_one_step_parity(gpu_lib, scheme, k, dtype):
    w = weibel_small(nx=32, ny=64, ppc=5, seed=21)
    degree = 3
    o = make_oracle(w, degree, scheme, k)
    ctx = make_gpu(w, degree, scheme, dtype, bdf_order=k)
    tol = DT_TOL[dtype]
    o.deposit()
    o.solve()
    pic.deposit_current(ctx)
    pic.field_solve(ctx)
    F = pic.get_field(ctx, pic.FIELD_MESH).cpu().numpy()
    for s in range(12):
        assert rel(F[s], o.fields[s]) <= tol, (s, rel(F[s], o.fields[s]))
    H = pic.get_history(ctx).cpu().numpy()
    Ho = hist_to_flat(o.p, o.hist)
    assert H.shape == Ho.shape
    for f in range(H.shape[0]):
        if np.abs(Ho[f]).max() > 0:
            assert rel(H[f], Ho[f]) <= tol, (f, rel(H[f], Ho[f]))
        else:
            assert np.abs(H[f]).max() == 0
    o.gather_push()
    pic.gather_push(ctx)
    errs, bad = compare_particles(gpu_parts(ctx), o.part, w["lx"], w["ly"], tol)
    assert not bad, errs


@pytest.mark.parametrize("scheme,k", SCHEMES)
def test_trajectory_parity_f64(gpu_lib, scheme, k):
    """Cold start, 30 steps through step() (fused path), float64 throughout."""
    w = cloud_small()
    o = make_oracle(w, 2, scheme, k)
    ctx = make_gpu(w, 2, scheme, "f64", bdf_order=k)
    for chunk in range(3):
        o.step(10)
        pic.step(ctx, 10)
        errs, bad = compare_particles(gpu_parts(ctx), o.part, w["lx"], w["ly"], 1e-10)
        assert not bad, (chunk, errs)
    H = pic.get_history(ctx).cpu().numpy()
    Ho = hist_to_flat(o.p, o.hist)
    assert rel(H, Ho) <= 1e-10


def test_fused_step_equals_unfused(gpu_lib):
    w = weibel_small(nx=64, ny=32, ppc=9, seed=5)
    a = make_gpu(w, 3, "bdf", "f64", bdf_order=2)
    b = make_gpu(w, 3, "bdf", "f64", bdf_order=2, flags=pic.FLAG_UNFUSED_STEP)
    pic.step(a, 12)
    for _ in range(12):
        pic.deposit_current(b)
        pic.field_solve(b)
        pic.gather_push(b)
    pa, pb = gpu_parts(a), gpu_parts(b)
    for key in pa:
        assert rel(pa[key], pb[key]) <= 1e-12, key


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_tiled_equals_untiled(gpu_lib, dtype, tol):
    """The tile-sorted LDS path and the plain global-atomic path agree."""
    w = weibel_small(nx=64, ny=32, ppc=9, seed=6)
    a = make_gpu(w, 3, "bdf", dtype, bdf_order=2)
    b = make_gpu(w, 3, "bdf", dtype, bdf_order=2, flags=pic.FLAG_NO_SORT)
    pic.step(a, 10)
    pic.step(b, 10)
    pa, pb = gpu_parts(a), gpu_parts(b)
    for key in pa:
        assert rel(pa[key], pb[key]) <= tol, (key, rel(pa[key], pb[key]))


def test_drift_beyond_slack_uses_global_path(gpu_lib):
    """A fast drift with a long sort interval moves particles out of their tile
    window; results must not change."""
    w = workloads.cloud(nx=32, ny=32, ppc=6, seed=8, drift=3.0, vth=0.2)
    o = make_oracle(w, 3, "bdf", 2)
    ctx = make_gpu(w, 3, "bdf", "f64", bdf_order=2, sort_interval=40)
    o.step(30)
    pic.step(ctx, 30)
    errs, bad = compare_particles(gpu_parts(ctx), o.part, w["lx"], w["ly"], 1e-10)
    assert not bad, errs


@pytest.mark.parametrize("scheme,k", [("bdf", 2), ("cdf2", 2), ("dirk2", 2)])
def test_f32_step_from_oracle_state(gpu_lib, scheme, k):
    """float32: run the oracle 8 steps, load its state into the GPU, compare one step."""
    w = weibel_small(nx=64, ny=64, ppc=4, seed=31)
    o = make_oracle(w, 3, scheme, k)
    o.step(8)
    ctx = make_gpu(w, 3, scheme, "f32", bdf_order=k)
    set_gpu_parts(ctx, o.part)
    pic.set_history(ctx, torch.as_tensor(hist_to_flat(o.p, o.hist)))
    o.step(1)
    pic.step(ctx, 1)
    errs, bad = compare_particles(gpu_parts(ctx), o.part, w["lx"], w["ly"], 1e-4)
    assert not bad, errs
    assert rel(pic.get_history(ctx).cpu().numpy(), hist_to_flat(o.p, o.hist)) <= 1e-4


@pytest.mark.parametrize("scheme,k", SCHEMES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gpu_invariants(gpu_lib, scheme, k, dtype):
    """Gauge residual at round-off every step (Sec. 3 theorems); Gauss for BDF/CDF."""
    w = cloud_small(nx=64, ny=32, ppc=4, seed=41)
    ctx = make_gpu(w, 2, scheme, dtype, bdf_order=k)
    for _ in range(5):
        pic.step(ctx, 4)
        d = pic.diagnostics(ctx)
        assert d["gauge_l2"] <= 1e3 * EPS * d["gauge_scale"], d
        assert abs(d["charge"]) <= 1e3 * EPS * d["gauss_scale"], d
        assert d["nonfinite"] == 0
        if scheme != "dirk2":
            assert d["gauss_l2"] <= 1e3 * EPS * d["gauss_scale"], d


def test_diagnostics_match_oracle(gpu_lib):
    w = cloud_small(seed=43)
    for scheme, k in SCHEMES:
        o = make_oracle(w, 2, scheme, k)
        ctx = make_gpu(w, 2, scheme, "f64", bdf_order=k)
        o.step(6)
        pic.step(ctx, 6)
        dg = pic.diagnostics(ctx)
        do = odiag.residuals(o)
        for key in ("gauge_scale", "gauss_scale", "energy"):
            assert rel(dg[key], do[key]) <= 1e-9, (scheme, key, dg[key], do[key])
        if scheme == "dirk2":
            assert rel(dg["gauss_l2"], do["gauss_l2"]) <= 1e-9


def test_history_roundtrip(gpu_lib):
    w = cloud_small(seed=44)
    o = make_oracle(w, 2, "cdf2")
    o.step(3)
    ctx = make_gpu(w, 2, "cdf2", "f64")
    Ho = hist_to_flat(o.p, o.hist)
    pic.set_history(ctx, torch.as_tensor(Ho))
    assert rel(pic.get_history(ctx).cpu().numpy(), Ho) == 0.0


# ---------------------------------------------------------------------------
# edge cases

def test_empty_particle_set(gpu_lib):
    w = cloud_small()
    w = dict(w, x=w["x"][:0], y=w["y"][:0], P=w["P"][:0])
    ctx = make_gpu(w, 2, "bdf", "f64", bdf_order=2, max_particles=16)
    pic.step(ctx, 3)
    d = pic.diagnostics(ctx)
    assert d["gauge_l2"] == 0.0 and d["energy"] == 0.0


def test_single_particle_and_seam_positions(gpu_lib):
    w = cloud_small()
    L = w["lx"]
    x = np.array([0.0, L * (1 - 1e-16), L - 1e-12, 0.5 * L, 1e-300])
    y = np.array([L * (1 - 1e-16), 0.0, 1e-14, 0.25 * L, L / 3])
    P = np.array([[-0.3, 0.2, 0.1], [0.4, -0.1, 0.0], [0.0, 0.0, 0.5], [0.3, 0.3, 0.3],
                  [-0.9, 0.0, 0.0]]) * w["m"]
    w = dict(w, x=x, y=y, P=P)
    for scheme, k in SCHEMES:
        o = make_oracle(w, 3, scheme, k)
        ctx = make_gpu(w, 3, scheme, "f64", bdf_order=k)
        o.step(5)
        pic.step(ctx, 5)
        errs, bad = compare_particles(gpu_parts(ctx), o.part, L, w["ly"], 1e-10)
        assert not bad, (scheme, errs)


def test_minimum_grid_and_phase_errors(gpu_lib):
    w = weibel_small(nx=8, ny=8, ppc=3, seed=3)
    o = make_oracle(w, 3, "bdf", 2)
    ctx = make_gpu(w, 3, "bdf", "f64", bdf_order=2)
    with pytest.raises(pic.PicError):
        pic.field_solve(ctx)        # out of order: needs DEPOSITED
    with pytest.raises(pic.PicError):
        pic.gather_push(ctx)
    o.step(4)
    pic.step(ctx, 4)
    errs, bad = compare_particles(gpu_parts(ctx), o.part, w["lx"], w["ly"], 1e-10)
    assert not bad, errs


def test_nonfinite_detected(gpu_lib):
    w = cloud_small()
    ctx = make_gpu(w, 2, "bdf", "f64", bdf_order=1)
    a = pic.get_particles(ctx)
    a[2, 7] = float("nan")
    pic.set_particles(ctx, a)
    with pytest.raises(pic.PicError) as e:
        pic.diagnostics(ctx)
    assert e.value.status == 6
    assert pic.diagnostics(ctx, allow_nonfinite=True)["nonfinite"] >= 1


# ---------------------------------------------------------------------------
# full size of the 128 x 128, 64 particles/cell anisotropic workload

def test_full_size_weibel_one_step_f32(gpu_lib):
    w = workloads.make("weibel128")
    o = make_oracle(w, 3, "bdf", 2)
    ctx = make_gpu(w, 3, "bdf", "f32", bdf_order=2)
    o.step(2)
    pic.step(ctx, 2)
    gp = gpu_parts(ctx)
    errs, bad = compare_particles(gp, o.part, w["lx"], w["ly"], 1e-4)
    assert not bad, errs
    d = pic.diagnostics(ctx)
    assert d["gauge_l2"] <= 1e3 * EPS * d["gauge_scale"]


@pytest.mark.parametrize("scheme,k", [("bdf", 2), ("cdf2", 2), ("dirk2", 2), ("dirk3", 2)])
def test_graph_replay_matches_oracle_and_direct(gpu_lib, scheme, k):
    """step() replays captured HIP graphs for long calls; results are those of
    direct launches and of the oracle."""
    w = cloud_small(seed=51)
    o = make_oracle(w, 2, scheme, k)
    g = make_gpu(w, 2, scheme, "f64", bdf_order=k)
    d = make_gpu(w, 2, scheme, "f64", bdf_order=k, flags=pic.FLAG_NO_GRAPH)
    assert pic.graph_period(g) > 0 and pic.graph_period(d) == 0
    # uneven call lengths: capture, replay, remainders, and calls that start
    # at another phase of the captured period (direct steps up to it, then
    # replays)
    for n in (40, 7, 25, 31, 3, 19):
        o.step(n)
        pic.step(g, n)
        pic.step(d, n)
    pg, pd = gpu_parts(g), gpu_parts(d)
    for key in pg:
        assert rel(pg[key], pd[key]) <= 1e-12, key
    errs, bad = compare_particles(pg, o.part, w["lx"], w["ly"], 1e-10)
    assert not bad, errs
    assert rel(pic.get_history(g).cpu().numpy(), hist_to_flat(o.p, o.hist)) <= 1e-10


def test_reload_at_every_phase_of_the_sort_cycle(gpu_lib):
    """Loading particles again after k steps -- whichever pass of the sort
    cycle came last, including one that already counted cells for a sort that
    then never runs -- gives the same run as a fresh context (up to the
    rounding order of the float64 deposit atomics)."""
    w = cloud_small(seed=61)
    fresh = make_gpu(w, 3, "bdf", "f64", bdf_order=2)
    pic.step(fresh, 9)
    ref = gpu_parts(fresh)
    data = (torch.as_tensor(w["x"], device=fresh.device), torch.as_tensor(w["y"], device=fresh.device),
            torch.as_tensor(np.ascontiguousarray(w["P"].T), device=fresh.device))
    for k in range(1, 14):
        g = make_gpu(w, 3, "bdf", "f64", bdf_order=2)
        pic.step(g, k)
        pic.init_particles(g, *data)
        pic.step(g, 9)
        got = gpu_parts(g)
        errs, bad = compare_particles(got, ref, w["lx"], w["ly"], 1e-12)
        assert not bad, (k, errs)
        g.close()


@pytest.mark.parametrize("degree", [4, 5])
@pytest.mark.parametrize("scheme,k", [("bdf", 2), ("dirk2", 2)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("flags", [0, pic.FLAG_NO_SORT])
def test_quartic_quintic_trajectory(gpu_lib, degree, scheme, k, dtype, flags):
    """Quartic and quintic splines (the higher-order weighting of the DIRK-2
    study, Sec. 5.1) through step(), tiled and untiled, against the oracle."""
    w = weibel_small(nx=32, ny=32, ppc=5, seed=80 + degree)
    o = make_oracle(w, degree, scheme, k)
    g = make_gpu(w, degree, scheme, dtype, bdf_order=k, flags=flags)
    for n in (1, 12):
        o.step(n)
        pic.step(g, n)
    tol = DT_TOL[dtype]
    errs, bad = compare_particles(gpu_parts(g), o.part, w["lx"], w["ly"], tol)
    assert not bad, errs
    assert rel(pic.get_history(g).cpu().numpy(), hist_to_flat(o.p, o.hist)) <= tol
    g.close()


def test_sort_interval_follows_inplane_speed(gpu_lib):
    """With sort_interval 0 the interval comes from the loaded particles'
    largest in-plane velocity: particles at rest get three times the speed-of-
    light interval, particles at 0.95c in x get the speed-of-light one (the graph
    period, two sort intervals rounded to the history rings, shows it); the
    slow run still matches the oracle."""
    w = cloud_small(seed=71)
    cold = dict(w, P=0.0 * w["P"])
    hot = dict(w, P=np.zeros_like(w["P"]))
    hot["P"][:, 0] = w["m"] * 0.95 / np.sqrt(1.0 - 0.95 ** 2)      # u_x for v_x = 0.95c
    gc = make_gpu(cold, 2, "bdf", "f64", bdf_order=2)
    gh = make_gpu(hot, 2, "bdf", "f64", bdf_order=2)
    # speed-of-light interval: slack 3 cells / (c dt / dx) = 6 steps here
    assert pic.graph_period(gh) == 12 and pic.graph_period(gc) == 36, (pic.graph_period(gh), pic.graph_period(gc))
    o = make_oracle(hot, 2, "bdf", 2)
    o.step(30)
    pic.step(gh, 30)
    errs, bad = compare_particles(gpu_parts(gh), o.part, w["lx"], w["ly"], 1e-10)
    assert not bad, errs
