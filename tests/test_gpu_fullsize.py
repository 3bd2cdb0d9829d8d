"""Full-size checks at the workload sizes the benchmark runs.

The 512 x 512, 256 particles/cell case (67,108,864 float32 particles, cubic,
DIRK-2 and CDF-2): from the original inputs, the oracle computes outputs one
by one -- J at sampled nodes (the definition summed over all particles) and
the first update's spectral history at sampled modes (the direct Fourier sum
of the deposit, then the per-mode stepper update); over the full 100 steps it
shadow-steps (the GPU state at steps 49 and 99 loaded into the oracle, one
step of each compared: the whole spectral history and a seeded sample of
1,048,576 particles).  Invariants that hold at any size: gauge residual at
round-off, zero net charge, finite state, |v| < c.

The 128 x 128 / 1,048,576-particle case runs through step() with HIP graph
replay (the launch configuration bench.py times): invariants over 30 steps,
and in float64 the graph-replayed run equals direct launches.
"""

import numpy as np
import pytest
import torch

from oracle import pic as opic
from paper_2410_18414_amd import pic, workloads
from pic_harness import compare_particles, hist_to_flat, make_gpu, oracle_params, rel

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def big():
    import time
    t0 = time.time()
    w = workloads.make("weibel512")
    assert len(w["x"]) == 512 * 512 * 256
    print("generated 67M particles in %.0f s" % (time.time() - t0), flush=True)
    p = oracle_params(w, 3, "dirk2")
    part = opic.init_particles(p, w["x"], w["y"], w["P"])
    x1, y1 = opic.position_update(p, part["x"], part["y"], part["v"])
    nodes = [(0, 0), (511, 511), (256, 100), (37, 400), (510, 1), (300, 0)]
    modes = [(0, 0), (1, 0), (3, 7), (40, 500), (256, 255)]
    Jn = opic.current_at_nodes(p, x1, y1, part["v"], nodes)
    print("oracle J at %d nodes after %.0f s" % (len(nodes), time.time() - t0), flush=True)
    Jm = opic.current_modes(p, x1, y1, part["v"], modes)
    print("oracle J^ at %d modes after %.0f s" % (len(modes), time.time() - t0), flush=True)
    return dict(w=w, nodes=nodes, modes=modes, Jn=Jn, Jm=Jm)


@pytest.mark.parametrize("scheme", ["dirk2", "cdf2"])
def test_512_first_step_sampled_and_invariants(gpu_lib, big, scheme):
    w = big["w"]
    p = oracle_params(w, 3, scheme)
    ctx = make_gpu(w, 3, scheme, "f32")
    print("512x512 / 67M particles,", scheme, flush=True)
    pic.deposit_current(ctx)
    J = pic.get_field(ctx, pic.FIELD_J).cpu().numpy()
    got = np.array([J[:, iy, ix] for ix, iy in big["nodes"]])
    assert rel(got, big["Jn"]) <= 1e-4, rel(got, big["Jn"])
    pic.field_solve(ctx)
    # expected first update at the sampled modes: the per-mode stepper update of
    # the sampled current spectrum (every other mode zero; the update is diagonal)
    Jh = np.zeros((3,) + p.spec_shape, np.complex128)
    for (kx, ky), val in zip(big["modes"], big["Jm"]):
        Jh[:, ky, kx] = val
    hist, _, _ = opic.field_update(p, opic.cold_history(p), Jh)
    ref = hist_to_flat(p, hist)
    H = pic.get_history(ctx).cpu().numpy()
    got = np.array([H[:, ky, kx] for kx, ky in big["modes"]])
    exp = np.array([ref[:, ky, kx] for kx, ky in big["modes"]])
    assert rel(got, exp) <= 1e-4, rel(got, exp)
    pic.gather_push(ctx)
    pic.step(ctx, 3)
    d = pic.diagnostics(ctx)
    assert d["nonfinite"] == 0
    assert d["gauge_l2"] <= 1e3 * EPS * d["gauge_scale"], d
    assert abs(d["charge"]) <= 1e-9 * abs(w["q"]) * len(w["x"]), d
    parts = pic.get_particles(ctx)
    assert torch.isfinite(parts).all()
    v2 = (parts[5:8] ** 2).sum(0)
    assert float(v2.max()) < 1.0
    ctx.close()


@pytest.mark.parametrize("scheme", ["dirk2", "cdf2"])
def test_512_100_steps_shadow_stepping(gpu_lib, big, scheme):
    """The 512x512 / 67,108,864-particle float32 workload over its full 100
    steps in the bench's launch configuration (step(), default tile plan).
    At steps 50 and 100 the oracle takes the GPU state (promoted to float64)
    and runs that step: the deposit over every particle, the field update and
    gradients, and the gather and push of a seeded sample of 1,048,576
    particles; the GPU's full spectral history (every field, every level) and
    the sampled particles must agree at the float32 tolerance (1e-4).  The
    gauge residual stays at round-off, the net charge at zero, |v| < c."""
    import time
    from pic_harness import flat_to_hist, shadow_step
    w = big["w"]
    n = len(w["x"])
    p = oracle_params(w, 3, scheme)
    g = make_gpu(w, 3, scheme, "f32")
    rng = np.random.default_rng(5120 + len(scheme))
    sample = np.sort(rng.choice(n, 1 << 20, replace=False))
    s_dev = torch.as_tensor(sample, device=g.device)
    t0 = time.time()
    done = 0
    for shadow_at in (50, 100):
        pic.step(g, shadow_at - 1 - done)
        a = pic.get_particles(g)
        x, y = a[0].cpu().numpy(), a[1].cpu().numpy()
        v = a[5:8].T.contiguous().cpu().numpy()
        P_s = a[2:5][:, s_dev].T.contiguous().cpu().numpy()
        vprev_s = a[8:11][:, s_dev].T.contiguous().cpu().numpy()
        del a
        hist = flat_to_hist(p, pic.get_history(g).cpu().numpy())
        pic.step(g, 1)
        done = shadow_at
        print("%s: GPU state exported at step %d (%.0f s)" % (scheme, shadow_at - 1, time.time() - t0), flush=True)
        ohist, opart = shadow_step(p, x, y, v, hist, sample, P_s, vprev_s)
        del x, y, v
        print("%s: oracle step %d done (%.0f s)" % (scheme, shadow_at, time.time() - t0), flush=True)
        b = pic.get_particles(g)[:, s_dev].cpu().numpy()
        gpart = dict(x=b[0], y=b[1], P=b[2:5].T, v=b[5:8].T, vprev=b[8:11].T)
        errs, bad = compare_particles(gpart, opart, w["lx"], w["ly"], 1e-4)
        assert not bad, (shadow_at, errs)
        H = pic.get_history(g).cpu().numpy()
        Ho = hist_to_flat(p, ohist)
        worst = max(rel(H[f], Ho[f]) for f in range(H.shape[0]))
        assert worst <= 1e-4, (shadow_at, worst)
        print("%s: step %d shadow ok, particles %s, history %.2e" % (scheme, shadow_at, errs, worst), flush=True)
    d = pic.diagnostics(g)
    assert d["nonfinite"] == 0
    assert d["gauge_l2"] <= 1e3 * EPS * d["gauge_scale"], d
    assert abs(d["charge"]) <= 1e-9 * abs(w["q"]) * n, d
    v2 = (pic.get_particles(g)[5:8] ** 2).sum(0)
    assert float(v2.max()) < 1.0
    g.close()


def test_128_graph_replay_invariants_and_direct_equality(gpu_lib):
    w = workloads.make("weibel128")
    ctx = make_gpu(w, 3, "bdf", "f32")
    pic.step(ctx, 30)  # captured once, then replayed
    d = pic.diagnostics(ctx)
    assert d["nonfinite"] == 0
    assert d["gauge_l2"] <= 1e3 * EPS * d["gauge_scale"], d
    assert abs(d["charge"]) <= 1e-9 * abs(w["q"]) * len(w["x"]), d
    ctx.close()
    # float64: the replayed graph equals direct launches
    g = make_gpu(w, 3, "bdf", "f64")
    n = make_gpu(w, 3, "bdf", "f64", flags=pic.FLAG_NO_GRAPH)
    pic.step(g, 30)
    pic.step(n, 30)
    a = pic.get_particles(g).cpu().numpy()
    b = pic.get_particles(n).cpu().numpy()
    for k in range(11):
        assert rel(a[k], b[k]) <= 1e-10, k
    assert rel(pic.get_history(g).cpu().numpy(), pic.get_history(n).cpu().numpy()) <= 1e-10


def test_cloud32_full_run_f64(gpu_lib):
    """The 32x32, 4 particles/cell drifting cloud (quadratic, BDF-1, float64)
    over its full 50 steps through graph-replayed step() against the oracle."""
    from pic_harness import compare_particles, gpu_parts, hist_to_flat, make_gpu, make_oracle
    w = workloads.make("cloud32")
    o = make_oracle(w, 2, "bdf", 1)
    g = make_gpu(w, 2, "bdf", "f64", bdf_order=1)
    o.step(50)
    pic.step(g, 50)
    errs, bad = compare_particles(gpu_parts(g), o.part, w["lx"], w["ly"], 1e-10)
    assert not bad, errs
    assert rel(pic.get_history(g).cpu().numpy(), hist_to_flat(o.p, o.hist)) <= 1e-10
    d = pic.diagnostics(g)
    assert d["gauge_l2"] <= 1e3 * EPS * d["gauge_scale"]
    g.close()


def test_weibel128_200_steps_shadow_stepping(gpu_lib):
    """The 128x128, 64 particles/cell float32 workload over its full 200 steps
    in the bench's launch configuration; every 20 steps the oracle is loaded
    with the GPU state (promoted to float64) and one step of each is compared
    (float32 parity 1e-4), and the gauge stays at round-off."""
    import time
    from pic_harness import compare_particles, gpu_parts, make_gpu, oracle_from_gpu
    w = workloads.make("weibel128")
    p = oracle_params(w, 3, "bdf", 2)
    g = make_gpu(w, 3, "bdf", "f32", bdf_order=2)
    t0 = time.time()
    done = 0
    while done < 200:
        pic.step(g, 19)
        o = oracle_from_gpu(p, g, w)
        o.step(1)
        pic.step(g, 1)
        done += 20
        errs, bad = compare_particles(gpu_parts(g), o.part, w["lx"], w["ly"], 1e-4)
        assert not bad, (done, errs)
        print("step %d shadow ok (%.0f s)" % (done, time.time() - t0), flush=True)
    d = pic.diagnostics(g)
    assert d["nonfinite"] == 0
    assert d["gauge_l2"] <= 1e3 * np.finfo(np.float64).eps * d["gauge_scale"], d
    g.close()


def test_full_ensemble_sampled(gpu_lib):
    """The 64-instance uneven ensemble (31M float32 particles) as the bench
    runs it (one context, graph-replayed step_batched): the four smallest
    instances against the oracle after 3 steps (1e-4), every instance's gauge
    residual at round-off."""
    import torch
    from pic_harness import compare_particles, gpu_parts, make_oracle
    ws = workloads.ensemble()
    cfgs = [pic.make_config(w["nx"], w["ny"], w["lx"], w["ly"], w["dt"], degree=3, scheme="bdf", bdf_order=2,
                            dtype="f32", q=w["q"], m=w["m"], max_particles=len(w["x"])) for w in ws]
    b = pic.Context(cfgs)
    for i, w in enumerate(ws):
        pic.select_instance(b, i)
        pic.init_particles(b, torch.as_tensor(w["x"], device=b.device), torch.as_tensor(w["y"], device=b.device),
                           torch.as_tensor(np.ascontiguousarray(w["P"].T), device=b.device))
    pic.step_batched(b, 3)
    for i in np.argsort([len(w["x"]) for w in ws])[:4]:
        w = ws[i]
        o = make_oracle(w, 3, "bdf", 2)
        o.step(3)
        pic.select_instance(b, int(i))
        errs, bad = compare_particles(gpu_parts(b), o.part, w["lx"], w["ly"], 1e-4)
        assert not bad, (int(i), errs)
    for i in range(len(ws)):
        pic.select_instance(b, i)
        d = pic.diagnostics(b)
        assert d["nonfinite"] == 0 and d["gauge_l2"] <= 1e3 * EPS * d["gauge_scale"], (i, d)
    b.close()
