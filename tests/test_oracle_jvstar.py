"""Pins of the oracle's v*-in-J mode (CPU only).

Sec. 4.2 allows J^{n+1} to carry the push's extrapolated velocity
v* = 2 v^n - v^{n-1} instead of v^n (the positions still move with v^n; the
paper reports no visible difference in its tests).  Pinned here:

* the deposited J is the definition J(x_g) = sum_p q v*_p S(x_g - x_p^{n+1}),
  by brute force over periodic images with the spline written as its
  Cox-de Boor recursion, and its mesh integral is q sum_p v*_p (partition of
  unity), which tells v* apart from v^n and v^{n-1} once particles accelerate;
* the first step of a cold start (v^{-1} = v^0) equals the plain run exactly;
* the gauge residual stays at round-off under every stepper (rho follows from
  continuity with whatever J is deposited) and so does Gauss's law for BDF-k.
"""

import numpy as np
import pytest

from oracle import diagnostics, pic
from paper_2410_18414_amd import workloads

EPS = np.finfo(float).eps


def _cox_de_boor(m, t):
    """Centred cardinal B-spline of degree m by the Cox-de Boor recursion on
    the integer knots -(m+1)/2, ..., (m+1)/2."""
    t = np.asarray(t, np.float64) + (m + 1) / 2.0

    def N(i, k, s):
        if k == 0:
            return np.where((s >= i) & (s < i + 1), 1.0, 0.0)
        return ((s - i) / k) * N(i, k - 1, s) + ((i + k + 1 - s) / k) * N(i + 1, k - 1, s)
    return N(0, m, t)


def _state(scheme, jvstar, degree=2, k=2, steps=0, nx=16, ny=16, ppc=4, seed=51):
    w = workloads.cloud(nx=nx, ny=ny, ppc=ppc, seed=seed, drift=0.3, vth=0.05)
    p = pic.Params(w["nx"], w["ny"], w["lx"], w["ly"], degree, scheme, w["dt"],
                   q=w["q"], m=w["m"], bdf_order=k, jvstar=jvstar)
    s = pic.State(p, w["x"], w["y"], w["P"])
    s.step(steps)
    return s


@pytest.mark.parametrize("degree", [1, 3])
def test_current_is_the_definition_with_vstar(degree):
    s = _state("bdf", True, degree=degree, nx=8, ny=8, ppc=1, steps=6)
    p, pt = s.p, s.part
    v, vp = pt["v"].copy(), pt["vprev"].copy()
    assert np.max(np.abs(v - vp)) > 1e-6 * np.max(np.abs(v))      # the particles accelerate
    s.deposit()
    vs = 2.0 * v - vp
    x, y = pt["x"], pt["y"]
    ref = np.zeros((3, p.ny, p.nx))
    for j in range(p.ny):
        for i in range(p.nx):
            wsum = 0.0
            for kx in (-1, 0, 1):
                for ky in (-1, 0, 1):
                    wx = _cox_de_boor(degree, (i * p.dx - x - kx * p.lx) / p.dx)
                    wy = _cox_de_boor(degree, (j * p.dy - y - ky * p.ly) / p.dy)
                    wsum = wsum + wx * wy
            ref[:, j, i] = p.q * (wsum[:, None] * vs).sum(axis=0) / (p.dx * p.dy)
    assert np.max(np.abs(s.J - ref)) <= 1e-12 * np.max(np.abs(ref))
    total = s.J.reshape(3, -1).sum(axis=1) * p.dx * p.dy
    want = p.q * vs.sum(axis=0)
    assert np.all(np.abs(total - want) <= 1e-12 * np.abs(p.q) * np.abs(vs).sum(axis=0))
    # v^n alone would give another total
    assert np.max(np.abs(total - p.q * v.sum(axis=0))) > 1e3 * np.max(np.abs(total - want))


@pytest.mark.parametrize("scheme", ["bdf", "cdf2", "dirk2"])
def test_first_step_equals_plain_run(scheme):
    a = _state(scheme, True, steps=1)
    b = _state(scheme, False, steps=1)
    for key in ("x", "y", "P", "v", "vprev"):
        assert np.array_equal(a.part[key], b.part[key]), key
    assert np.array_equal(a.J, b.J)


@pytest.mark.parametrize("scheme,k", [("bdf", 1), ("bdf", 2), ("bdf", 3), ("cdf2", 2),
                                      ("cdf2_semi", 2), ("dirk2", 2), ("dirk3", 2)])
def test_gauge_at_round_off(scheme, k):
    s = _state(scheme, True, k=k, steps=15)
    r = diagnostics.residuals(s)
    assert r["gauge_l2"] <= 1e3 * EPS * r["gauge_scale"], r
    if scheme == "bdf":
        assert r["gauss_l2"] <= 1e3 * EPS * r["gauss_scale"], r

