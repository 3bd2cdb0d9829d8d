"""GPU parity of the discrete adjoint (step_adjoint and friends) against the
autograd oracle, and of the full-size gradient against finite differences.

Reference values come from oracle/adjoint.py (torch CPU float64 autograd of
the oracle step), which the CPU suite pins to the numpy oracle and to finite
differences.  Tolerances: 1e-10 normwise relative (float64 parity), 1e-12 for
checkpointed vs store-all, 1e-6 for Richardson-extrapolated central
differences at the full 128 x 128, 64 particles/cell, 20-step size.
"""

import numpy as np
import pytest
import torch

from oracle import adjoint as oadj
from oracle import pic as opic
from paper_2410_18414_amd import workloads
from pic_harness import hist_to_flat, oracle_params, rel

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _weibel(nx=32, ny=32, ppc=4, seed=7, drift=0.1):
    return workloads.weibel(nx=nx, ny=ny, ppc=ppc, seed=seed, drift=drift)


def _ctx(pic, w, degree=3, bdf_order=2, flags=0, dtype="f64"):
    n = w["x"].shape[0]
    cfg = pic.make_config(w["nx"], w["ny"], w["lx"], w["ly"], w["dt"], degree=degree, scheme="bdf",
                          bdf_order=bdf_order, dtype=dtype, q=w["q"], m=w["m"], max_particles=n,
                          flags=flags | pic.FLAG_ADJOINT)
    return pic.Context(cfg)


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def _load_state(pic, ctx, w, s):
    """Put the oracle state s (particles + history) into the context."""
    pic.init_particles(ctx, _dev(w["x"]), _dev(w["y"]), _dev(w["P"].T))
    pt = s.part
    a = np.concatenate([pt["x"][None], pt["y"][None], pt["P"].T, pt["v"].T, pt["vprev"].T])
    pic.set_particles(ctx, _dev(a))
    pic.set_history(ctx, _dev(hist_to_flat(s.p, s.hist)))


def test_energy_seed_matches_oracle(gpu_lib):
    pic = gpu_lib
    w = _weibel(seed=21)
    p = oracle_params(w, 3, "bdf", 2)
    s = opic.State(p, w["x"], w["y"], w["P"])
    s.step(4)
    ctx = _ctx(pic, w)
    _load_state(pic, ctx, w, s)
    g = pic.adjoint_seed_energy(ctx, 1.0).cpu().numpy()
    ref = oadj.energy_hist_grad(p, s.hist)
    assert rel(g, ref) <= TOL
    g2 = pic.adjoint_seed_energy(ctx, -2.5).cpu().numpy()
    assert rel(g2, -2.5 * ref) <= TOL


@pytest.mark.parametrize("degree,bdf_order,flags", [
    (3, 2, 0), (3, 2, 1), (2, 2, 0), (1, 2, 0), (3, 1, 0), (3, 3, 0), (2, 1, 1)])
def test_one_adjoint_step_matches_oracle_vjp(gpu_lib, degree, bdf_order, flags):
    """lambda^n = (dS^{n+1}/dS^n)^T lambda^{n+1} for a random lambda^{n+1}
    (particles and every history level), from a state after three steps."""
    pic = gpu_lib
    w = _weibel(nx=32, ny=16, ppc=5, seed=30 + degree + 10 * bdf_order)
    p = oracle_params(w, degree, "bdf", bdf_order)
    s = opic.State(p, w["x"], w["y"], w["P"])
    s.step(3)
    rng = np.random.default_rng(degree * 7 + bdf_order)
    part = {k: s.part[k] for k in ("x", "y", "P", "v", "vprev")}
    lp = {k: rng.standard_normal(np.shape(part[k])) for k in part}
    flat = hist_to_flat(p, s.hist)
    lh = rng.standard_normal(flat.shape) + 1j * rng.standard_normal(flat.shape)
    ref_p, ref_h = oadj.step_vjp(p, part, s.hist, lp, lh)

    ctx = _ctx(pic, w, degree=degree, bdf_order=bdf_order, flags=flags)
    _load_state(pic, ctx, w, s)
    lam = _dev(np.concatenate([lp["x"][None], lp["y"][None], lp["P"].T, lp["v"].T, lp["vprev"].T]))
    lam_h = _dev(lh)
    pic.step_adjoint(ctx, lam, lam_h)
    out = lam.cpu().numpy()
    got = dict(x=out[0], y=out[1], P=out[2:5].T, v=out[5:8].T, vprev=out[8:11].T)
    for k in got:
        assert rel(got[k], ref_p[k]) <= TOL, (k, rel(got[k], ref_p[k]))
    assert rel(lam_h.cpu().numpy(), ref_h) <= TOL
    # the forward recompute leaves the context as after deposit_current + field_solve
    pic.gather_push(ctx)
    s.step(1)
    gp = pic.get_particles(ctx).cpu().numpy()
    assert rel(gp[2:5].T, s.part["P"]) <= TOL


@pytest.mark.parametrize("flags", [0, 1])
def test_gradient_matches_oracle_autograd(gpu_lib, flags):
    from paper_2410_18414_amd import adjoint
    pic = gpu_lib
    w = _weibel(nx=32, ny=32, ppc=4, seed=41)
    nsteps = 10
    p = oracle_params(w, 3, "bdf", 2)
    W_ref, gx_ref, gy_ref, gP_ref = oadj.loss_and_grad(p, w["x"], w["y"], w["P"], nsteps)
    ctx = _ctx(pic, w, flags=flags)
    x0 = _dev(w["x"]).requires_grad_()
    y0 = _dev(w["y"]).requires_grad_()
    P0 = _dev(w["P"].T).requires_grad_()
    W = adjoint.field_energy(ctx, x0, y0, P0, nsteps, every=5)
    W.backward()
    assert abs(W.item() - W_ref) <= 1e-12 * abs(W_ref)
    assert rel(x0.grad.cpu().numpy(), gx_ref) <= TOL
    assert rel(y0.grad.cpu().numpy(), gy_ref) <= TOL
    assert rel(P0.grad.cpu().numpy().T, gP_ref) <= TOL


def test_checkpointed_equals_store_all(gpu_lib):
    from paper_2410_18414_amd import adjoint
    pic = gpu_lib
    w = _weibel(nx=64, ny=32, ppc=6, seed=43)
    ctx = _ctx(pic, w)
    grads = {}
    for every in (1, 5, 3):
        x0 = _dev(w["x"]).requires_grad_()
        y0 = _dev(w["y"]).requires_grad_()
        P0 = _dev(w["P"].T).requires_grad_()
        adjoint.field_energy(ctx, x0, y0, P0, 12, every=every).backward()
        grads[every] = [t.grad.cpu().numpy() for t in (x0, y0, P0)]
    for every in (5, 3):
        for a, b in zip(grads[every], grads[1]):
            assert rel(a, b) <= 1e-12


def test_held_adjoint_equals_explicit_across_sorts(gpu_lib):
    """The particle adjoint held in slot order (permuted when a sort changes
    the order) equals the one passed in original order at every step, over a
    sweep whose states straddle several sorts (sort interval 2)."""
    pic = gpu_lib
    w = _weibel(nx=32, ny=32, ppc=4, seed=47)
    n = w["x"].shape[0]
    cfg = pic.make_config(w["nx"], w["ny"], w["lx"], w["ly"], w["dt"], degree=3, scheme="bdf", bdf_order=2,
                          dtype="f64", q=w["q"], m=w["m"], max_particles=n + 5, flags=pic.FLAG_ADJOINT,
                          sort_interval=2)
    ctx = pic.Context(cfg)
    pic.init_particles(ctx, _dev(w["x"]), _dev(w["y"]), _dev(w["P"].T))
    states = []
    for _ in range(7):
        states.append(pic.save_state(ctx))
        pic.step(ctx, 1)
    seed_h = pic.adjoint_seed_energy(ctx, 1.0)
    g = torch.Generator().manual_seed(5)
    lam0 = torch.randn((11, n), generator=g, dtype=torch.float64).to("cuda")
    lam_e, h_e = lam0.clone(), seed_h.clone()
    for st in reversed(states):
        pic.load_state(ctx, st)
        pic.step_adjoint(ctx, lam_e, h_e)
    pic.adjoint_set_particles(ctx, lam0)
    h_h = seed_h.clone()
    for st in reversed(states):
        pic.load_state(ctx, st)
        pic.step_adjoint(ctx, None, h_h)
    lam_h = pic.adjoint_get_particles(ctx)
    assert rel(lam_h.cpu().numpy(), lam_e.cpu().numpy()) <= 1e-12
    assert rel(h_h.cpu().numpy(), h_e.cpu().numpy()) <= 1e-12
    # nothing held for another particle count
    pic.init_particles(ctx, _dev(w["x"][:-3]), _dev(w["y"][:-3]), _dev(w["P"][:-3].T))
    with pytest.raises(pic.PicError):
        pic.adjoint_get_particles(ctx)
    with pytest.raises(pic.PicError):
        pic.step_adjoint(ctx, None, h_h)


def test_step_adjoint_from_solved_state_equals_recompute(gpu_lib):
    """step_adjoint on a state saved after deposit_current + field_solve
    (phase SOLVED: nothing recomputed) equals step_adjoint on the state
    before them (phase READY: recomputed); a second step_adjoint on the same
    state is refused; the SOLVED state steps on like the context it was
    saved from."""
    pic = gpu_lib
    w = _weibel(nx=32, ny=32, ppc=4, seed=59)
    n = w["x"].shape[0]
    ctx = _ctx(pic, w)
    pic.init_particles(ctx, _dev(w["x"]), _dev(w["y"]), _dev(w["P"].T))
    pic.step(ctx, 3)
    ready = pic.save_state(ctx)
    pic.deposit_current(ctx)
    pic.field_solve(ctx)
    solved = pic.save_state(ctx)
    pic.gather_push(ctx)
    p_ref = pic.get_particles(ctx).cpu().numpy()
    g = torch.Generator().manual_seed(11)
    lam0 = torch.randn((11, n), generator=g, dtype=torch.float64).to("cuda")
    h0 = pic.adjoint_seed_energy(ctx, 1.0)
    h0 = h0 + torch.randn(h0.shape, generator=g, dtype=torch.complex128).to("cuda")
    pic.load_state(ctx, ready)
    lam_a, h_a = lam0.clone(), h0.clone()
    pic.step_adjoint(ctx, lam_a, h_a)
    with pytest.raises(pic.PicError) as e:
        pic.step_adjoint(ctx, lam0.clone(), h0.clone())
    assert e.value.status == 5
    pic.load_state(ctx, solved, trust_header=True)
    lam_b, h_b = lam0.clone(), h0.clone()
    pic.step_adjoint(ctx, lam_b, h_b)
    assert rel(lam_b.cpu().numpy(), lam_a.cpu().numpy()) <= 1e-12
    assert rel(h_b.cpu().numpy(), h_a.cpu().numpy()) <= 1e-12
    pic.load_state(ctx, solved)
    pic.gather_push(ctx)
    assert rel(pic.get_particles(ctx).cpu().numpy(), p_ref) <= 1e-14


def test_gradient_with_particles_past_their_windows(gpu_lib):
    """Counter-streaming particles at |v_x| up to about 0.75 c (0.37 cells a
    step) with a sort every 10 position updates: before each sort nearly
    every particle has moved more than the 3-cell slack of its tile window,
    so the forward passes, the replays and the adjoint passes take their
    global paths for them; the gradient still matches the oracle's, with
    checkpoints every 4 steps and storing every state."""
    from paper_2410_18414_amd import adjoint
    pic = gpu_lib
    w = _weibel(nx=32, ny=32, ppc=4, seed=53, drift=0.9)
    nsteps, every, interval = 12, 4, 10
    u = w["P"] / w["m"]
    vx = np.abs(u[:, 0]) / np.sqrt(1.0 + (u * u).sum(axis=1))
    dx = w["lx"] / w["nx"]
    assert vx.max() * w["dt"] * (interval + 1) / dx > 3.0  # past the slack before a sort is taken
    p = oracle_params(w, 3, "bdf", 2)
    W_ref, gx_ref, gy_ref, gP_ref = oadj.loss_and_grad(p, w["x"], w["y"], w["P"], nsteps)
    n = w["x"].shape[0]
    cfg = pic.make_config(w["nx"], w["ny"], w["lx"], w["ly"], w["dt"], degree=3, scheme="bdf", bdf_order=2,
                          dtype="f64", q=w["q"], m=w["m"], max_particles=n, flags=pic.FLAG_ADJOINT,
                          sort_interval=interval)
    ctx = pic.Context(cfg)
    for ev in (every, 1):
        x0 = _dev(w["x"]).requires_grad_()
        y0 = _dev(w["y"]).requires_grad_()
        P0 = _dev(w["P"].T).requires_grad_()
        W = adjoint.field_energy(ctx, x0, y0, P0, nsteps, every=ev)
        W.backward()
        assert abs(W.item() - W_ref) <= 1e-12 * abs(W_ref)
        assert rel(x0.grad.cpu().numpy(), gx_ref) <= TOL
        assert rel(y0.grad.cpu().numpy(), gy_ref) <= TOL
        assert rel(P0.grad.cpu().numpy().T, gP_ref) <= TOL


def test_adjoint_rejects_unsupported_contexts(gpu_lib):
    pic = gpu_lib
    w = _weibel(nx=16, ny=16, ppc=2, seed=5)
    n = w["x"].shape[0]
    hist = torch.zeros((18, 16, 9), dtype=torch.complex128, device="cuda")
    lam = torch.zeros((11, n), dtype=torch.float64, device="cuda")
    # no PIC_FLAG_ADJOINT
    cfg = pic.make_config(16, 16, w["lx"], w["ly"], w["dt"], degree=3, scheme="bdf", bdf_order=2,
                          dtype="f64", q=w["q"], m=w["m"], max_particles=n)
    ctx = pic.Context(cfg)
    pic.init_particles(ctx, _dev(w["x"]), _dev(w["y"]), _dev(w["P"].T))
    with pytest.raises(pic.PicError) as e:
        pic.step_adjoint(ctx, lam, hist)
    assert e.value.status == 2
    # float32 particles
    ctx = _ctx(pic, w, dtype="f32")
    pic.init_particles(ctx, _dev(w["x"]), _dev(w["y"]), _dev(w["P"].T))
    with pytest.raises(pic.PicError) as e:
        pic.step_adjoint(ctx, lam, hist)
    assert e.value.status == 2
    # quartic spline (the adjoint covers degrees 1..3)
    cfg = pic.make_config(16, 16, w["lx"], w["ly"], w["dt"], degree=4, scheme="bdf", bdf_order=2,
                          dtype="f64", q=w["q"], m=w["m"], max_particles=n, flags=pic.FLAG_ADJOINT)
    ctx = pic.Context(cfg)
    pic.init_particles(ctx, _dev(w["x"]), _dev(w["y"]), _dev(w["P"].T))
    with pytest.raises(pic.PicError) as e:
        pic.step_adjoint(ctx, lam, hist)
    assert e.value.status == 2
    # wrong phase: after deposit_current
    ctx = _ctx(pic, w)
    pic.init_particles(ctx, _dev(w["x"]), _dev(w["y"]), _dev(w["P"].T))
    pic.deposit_current(ctx)
    with pytest.raises(pic.PicError) as e:
        pic.step_adjoint(ctx, lam, hist)
    assert e.value.status == 5


def _theta_momenta(w_pos_xi, m, ud, a, vth=0.3):
    """P0(u_d, a) of the anisotropic workload as a torch expression."""
    xi = w_pos_xi
    n = xi.shape[0]
    sgn = torch.where(torch.arange(n, device=xi.device) % 2 == 0, 1.0, -1.0).to(torch.float64)
    ux = sgn * ud + vth / torch.sqrt(a) * xi[:, 0]
    uy = vth / torch.sqrt(a) * xi[:, 1]
    uz = vth * xi[:, 2] + 0.0 * a
    return m * torch.stack([ux, uy, uz])


def test_full_size_gradient_matches_finite_differences(gpu_lib):
    """d W / d(u_d, a) through 20 BDF-2 steps of the 128 x 128, 64
    particles/cell anisotropic workload with drift (float64, checkpoints every
    5 steps) against Richardson-extrapolated central differences."""
    from paper_2410_18414_amd import adjoint
    pic = gpu_lib
    w = workloads.make("weibel128-drift")
    nsteps = w["steps"]
    pos, xi = workloads.weibel_normals(128, 128, 64, 1005)
    xi_t = _dev(xi)
    # the generator's own momenta are reproduced by the torch expression
    P_chk = _theta_momenta(xi_t, w["m"], torch.tensor(0.1, dtype=torch.float64, device="cuda"),
                           torch.tensor(25.0, dtype=torch.float64, device="cuda"))
    assert rel(P_chk.cpu().numpy().T, w["P"]) <= 1e-14
    ctx = _ctx(pic, w)
    x0, y0 = _dev(w["x"]), _dev(w["y"])
    ud = torch.tensor(0.1, dtype=torch.float64, device="cuda", requires_grad=True)
    a = torch.tensor(25.0, dtype=torch.float64, device="cuda", requires_grad=True)
    W = adjoint.field_energy(ctx, x0, y0, _theta_momenta(xi_t, w["m"], ud, a), nsteps, every=5)
    W.backward()
    grad = {"ud": ud.grad.item(), "a": a.grad.item()}
    print("W", W.item(), "grad", grad, flush=True)

    def W_at(udv, av):
        with torch.no_grad():
            P0 = _theta_momenta(xi_t, w["m"], torch.tensor(udv, dtype=torch.float64, device="cuda"),
                                torch.tensor(av, dtype=torch.float64, device="cuda"))
            return adjoint.field_energy(ctx, x0, y0, P0, nsteps, every=nsteps).item()

    for name, base, h in (("ud", 0.1, 1e-5), ("a", 25.0, 2.5e-3)):
        est = {}
        for hh in (h, h / 2):
            plus = W_at(base + hh, 25.0) if name == "ud" else W_at(0.1, base + hh)
            minus = W_at(base - hh, 25.0) if name == "ud" else W_at(0.1, base - hh)
            est[hh] = (plus - minus) / (2 * hh)
        rich = (4 * est[h / 2] - est[h]) / 3
        print(name, "adjoint", grad[name], "fd", est, "richardson", rich, flush=True)
        assert abs(rich - grad[name]) <= 1e-6 * abs(grad[name]), (name, rich, grad[name])
