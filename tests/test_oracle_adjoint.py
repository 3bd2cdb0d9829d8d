"""Pins of the autograd reference gradient (CPU only).

* Its torch forward equals the numpy oracle (oracle/pic.py) step by step.
* Its gradient equals central finite differences of the same forward, with a
  Richardson check on the step size.
* Its loss equals the oracle diagnostics' field energy.
"""

import numpy as np
import pytest
import torch

from oracle import adjoint, diagnostics, pic
from paper_2410_18414_amd import workloads


def small(seed=3, nx=16, ny=8, ppc=3, drift=0.2):
    w = workloads.weibel(nx=nx, ny=ny, ppc=ppc, seed=seed, drift=drift)
    p = pic.Params(w["nx"], w["ny"], w["lx"], w["ly"], 3, "bdf", w["dt"], q=w["q"], m=w["m"],
                   bdf_order=2)
    return w, p


def test_torch_forward_equals_numpy_oracle():
    w, p = small()
    pr = adjoint.Problem(p)
    out = adjoint.run(pr, torch.tensor(w["x"]), torch.tensor(w["y"]), torch.tensor(w["P"]), 6)
    s = pic.State(p, w["x"], w["y"], w["P"])
    s.step(6)
    np.testing.assert_allclose(out["P"].numpy(), s.part["P"], rtol=0, atol=1e-14 * np.abs(s.part["P"]).max())
    np.testing.assert_allclose(out["v"].numpy(), s.part["v"], rtol=0, atol=1e-13)
    np.testing.assert_allclose(out["x"].numpy(), s.part["x"], rtol=0, atol=1e-13)
    W = float(adjoint.energy(pr, out["hist"]))
    assert abs(W - diagnostics.residuals(s)["energy"]) <= 1e-12 * abs(W)


def test_gradient_matches_central_differences():
    w, p = small(seed=5)
    nsteps = 5
    W, gx, gy, gP = adjoint.loss_and_grad(p, w["x"], w["y"], w["P"], nsteps)
    rng = np.random.default_rng(0)
    # directional derivative along random directions in P and in x
    for which in ("P", "x"):
        d = rng.standard_normal(w[which].shape)
        g = gP if which == "P" else gx
        scale = np.abs(w["P"]).max() if which == "P" else p.dx
        est = {}
        for h in (1e-3, 5e-4):
            plus, minus = dict(w), dict(w)
            plus[which] = w[which] + h * scale * d
            minus[which] = w[which] - h * scale * d
            est[h] = (adjoint.loss(p, plus["x"], plus["y"], plus["P"], nsteps)
                      - adjoint.loss(p, minus["x"], minus["y"], minus["P"], nsteps)) / (2 * h * scale)
        exact = float(np.sum(g * d))
        rich = (4 * est[5e-4] - est[1e-3]) / 3
        assert abs(rich - exact) <= 1e-6 * abs(exact), (which, rich, exact, est)


def _numpy_step(p, part, hist):
    """One step of the numpy oracle from an explicit state (copies its inputs)."""
    import copy
    s = pic.State(p, part["x"], part["y"], part["P"])
    s.part = {k: np.array(v, copy=True) for k, v in part.items()}
    s.hist = copy.deepcopy(hist)
    s.step(1)
    return s.part, s.hist


def _flat(h):
    out = list(h["rho"]) + list(h["phi"])
    for A in h["A"]:
        out += [A[0], A[1], A[2]]
    return np.stack(out)


def _pair(lp, lh, part, hist):
    tot = sum(np.sum(lp[k] * part[k]) for k in ("x", "y", "P", "v", "vprev"))
    return tot + np.sum((np.conj(lh) * _flat(hist)).real)


def test_step_vjp_dot_product_against_numpy_oracle():
    """<lambda, (S(s + h d) - S(s - h d)) / 2h> = <VJP(lambda), d> with the
    numpy oracle's step on the left and the autograd VJP on the right."""
    w, p = small(seed=9)
    s = pic.State(p, w["x"], w["y"], w["P"])
    s.step(3)  # a state with non-trivial history and v^n != v^{n-1}
    part = {k: s.part[k] for k in ("x", "y", "P", "v", "vprev")}
    rng = np.random.default_rng(4)
    flat0 = _flat(s.hist)
    lp = {k: rng.standard_normal(np.shape(part[k])) for k in part}
    lh = rng.standard_normal(flat0.shape) + 1j * rng.standard_normal(flat0.shape)
    gp, gh = adjoint.step_vjp(p, part, s.hist, lp, lh)
    # direction: particles and history (history perturbation on every level)
    dp = {k: rng.standard_normal(np.shape(part[k])) for k in part}
    dp["x"] *= p.dx
    dp["y"] *= p.dy
    for k in ("P", "v", "vprev"):
        dp[k] *= np.abs(part[k]).max()
    dh_scale = np.abs(flat0).max()
    dh = dh_scale * (rng.standard_normal(flat0.shape) + 1j * rng.standard_normal(flat0.shape))

    def perturbed(h):
        pt = {k: part[k] + h * dp[k] for k in part}
        hh = {"rho": [], "phi": [], "A": []}
        f = 0
        for lvl in s.hist["rho"]:
            hh["rho"].append(lvl + h * dh[f]); f += 1
        for lvl in s.hist["phi"]:
            hh["phi"].append(lvl + h * dh[f]); f += 1
        for lvl in s.hist["A"]:
            hh["A"].append(lvl + h * dh[f:f + 3]); f += 3
        return _numpy_step(p, pt, hh)

    est = {}
    for h in (1e-4, 5e-5):
        a = perturbed(h)
        b = perturbed(-h)
        est[h] = (_pair(lp, lh, *a) - _pair(lp, lh, *b)) / (2 * h)
    rich = (4 * est[5e-5] - est[1e-4]) / 3
    exact = sum(np.sum(gp[k] * dp[k]) for k in dp) + np.sum((np.conj(gh) * dh).real)
    assert abs(rich - exact) <= 1e-7 * abs(exact), (rich, exact, est)


def test_energy_history_gradient_against_differences():
    w, p = small(seed=11)
    s = pic.State(p, w["x"], w["y"], w["P"])
    s.step(4)
    g = adjoint.energy_hist_grad(p, s.hist)
    flat0 = _flat(s.hist)
    rng = np.random.default_rng(1)
    dh = np.abs(flat0).max() * (rng.standard_normal(flat0.shape) + 1j * rng.standard_normal(flat0.shape))
    pr = adjoint.Problem(p)
    k = p.bdf_order

    def W(h):
        f = flat0 + h * dh
        hh = dict(rho=[torch.tensor(f[j]) for j in range(k)],
                  phi=[torch.tensor(f[k + j]) for j in range(2 * k)],
                  A=[torch.tensor(f[3 * k + 3 * j:3 * k + 3 * j + 3]) for j in range(2 * k)])
        return float(adjoint.energy(pr, hh))

    h = 1e-3  # W is quadratic in the history: central differences are exact up to rounding
    est = (W(h) - W(-h)) / (2 * h)
    exact = np.sum((np.conj(g) * dh).real)
    assert abs(est - exact) <= 1e-9 * abs(exact)
    # only phi^n and A^{n..n-k} carry the energy
    assert np.all(g[:k] == 0) and np.all(g[k + 1:3 * k] == 0) and np.all(g[3 * k + 3 * (k + 1):] == 0)
