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
