"""Pins of the oracle's shape function, deposit and gather (CPU only).

The oracle writes M_m as a piecewise polynomial; here it is checked against
the Cox-de Boor recursion for cardinal B-splines (an independent definition),
against the spline's moment identities, and the deposit/gather against an
all-pairs brute force with explicit periodic images.
"""

import numpy as np
import pytest

from oracle import bspline, pic


def cox_de_boor(m, t):
    """Centred cardinal B-spline by the recursion
    N_1 = 1 on [0,1);  N_{k+1}(x) = (x N_k(x) + (k+1-x) N_k(x-1)) / k,
    M_m(t) = N_{m+1}(t + (m+1)/2)."""
    def N(k, x):
        if k == 1:
            return np.where((x >= 0) & (x < 1), 1.0, 0.0)
        return (x * N(k - 1, x) + (k - x) * N(k - 1, x - 1)) / (k - 1)
    t = np.asarray(t, float)
    return N(m + 1, t + (m + 1) / 2.0)


@pytest.mark.parametrize("m", [0, 1, 2, 3, 4, 5])
def test_spline_matches_cox_de_boor(m):
    t = np.linspace(-3.2, 3.2, 20001)
    np.testing.assert_allclose(bspline.M(m, t), cox_de_boor(m, t), atol=1e-14)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_spline_moments(m):
    rng = np.random.default_rng(0)
    xi = rng.uniform(-50, 50, 5000)
    g, w = bspline.stencil(m, xi)
    d = g - xi[:, None]
    np.testing.assert_allclose(w.sum(1), 1.0, atol=1e-14)           # partition of unity
    np.testing.assert_allclose((w * d).sum(1), 0.0, atol=1e-13)      # symmetric spline
    if m >= 2:   # polynomial reproduction up to degree m gives the exact 2nd moment
        np.testing.assert_allclose((w * d * d).sum(1), (m + 1) / 12.0, atol=1e-13)
    else:        # linear spline: discrete 2nd moment is delta (1 - delta)
        dl = xi - np.floor(xi)
        np.testing.assert_allclose((w * d * d).sum(1), dl * (1 - dl), atol=1e-13)


def brute_deposit(p, x, y, v):
    """Every node x every particle x periodic image, M by Cox-de Boor."""
    J = np.zeros((3, p.ny, p.nx))
    for j in range(p.ny):
        for i in range(p.nx):
            for n in range(x.shape[0]):
                s = 0.0
                for ix in (-1, 0, 1):
                    for iy in (-1, 0, 1):
                        tx = (i * p.dx - (x[n] + ix * p.lx)) / p.dx
                        ty = (j * p.dy - (y[n] + iy * p.ly)) / p.dy
                        s += cox_de_boor(p.degree, tx) * cox_de_boor(p.degree, ty)
                J[:, j, i] += p.q * v[n] * s / (p.dx * p.dy)
    return J


@pytest.mark.parametrize("m,nx,ny", [(1, 4, 4), (2, 4, 4), (3, 8, 6), (2, 5, 7), (4, 8, 6), (5, 8, 8)])
def test_deposit_brute_force(m, nx, ny):
    rng = np.random.default_rng(m * 100 + nx)
    p = pic.Params(nx, ny, 1.3, 0.9, m, "bdf", 0.01, q=-0.7)
    n = 7
    x = rng.uniform(0, p.lx, n)
    y = rng.uniform(0, p.ly, n)
    x[0] = 0.0
    y[1] = p.ly * (1 - 1e-15)
    v = rng.normal(0, 0.3, (n, 3))
    np.testing.assert_allclose(pic.deposit_current(p, x, y, v), brute_deposit(p, x, y, v),
                               rtol=0, atol=1e-12)


def test_deposit_total_current():
    """k = 0 mode: sum_g J dx dy = sum_p q v_p exactly (partition of unity)."""
    rng = np.random.default_rng(3)
    p = pic.Params(16, 8, 2.0, 1.0, 3, "bdf", 0.01, q=0.3)
    x = rng.uniform(0, p.lx, 500)
    y = rng.uniform(0, p.ly, 500)
    v = rng.normal(0, 0.3, (500, 3))
    J = pic.deposit_current(p, x, y, v)
    np.testing.assert_allclose(J.sum((1, 2)) * p.dx * p.dy, p.q * v.sum(0), atol=1e-13)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_gather_reproduces_linear_fields(m):
    """Symmetric B-spline interpolation reproduces constants and linear functions."""
    rng = np.random.default_rng(m)
    p = pic.Params(32, 16, 3.2, 1.6, m, "bdf", 0.01)
    x = rng.uniform(0.5, 2.5, 200)   # away from the periodic seam
    y = rng.uniform(0.4, 1.2, 200)
    X, Y = np.meshgrid(np.arange(p.nx) * p.dx, np.arange(p.ny) * p.dy)
    F = np.stack([np.ones_like(X), X, Y, 2.0 * X - 3.0 * Y + 1.0])
    g = pic.gather(p, F, x, y)
    np.testing.assert_allclose(g[:, 0], 1.0, atol=1e-14)
    np.testing.assert_allclose(g[:, 1], x, atol=1e-13)
    np.testing.assert_allclose(g[:, 2], y, atol=1e-13)
    np.testing.assert_allclose(g[:, 3], 2 * x - 3 * y + 1, atol=1e-13)


def test_gather_brute_force():
    rng = np.random.default_rng(9)
    p = pic.Params(6, 5, 1.2, 1.0, 3, "bdf", 0.01)
    F = rng.normal(size=(3, p.ny, p.nx))
    x = rng.uniform(0, p.lx, 5)
    y = rng.uniform(0, p.ly, 5)
    ref = np.zeros((5, 3))
    for n in range(5):
        for j in range(p.ny):
            for i in range(p.nx):
                s = 0.0
                for ix in (-1, 0, 1):
                    for iy in (-1, 0, 1):
                        s += (cox_de_boor(3, (i * p.dx - x[n] - ix * p.lx) / p.dx)
                              * cox_de_boor(3, (j * p.dy - y[n] - iy * p.ly) / p.dy))
                ref[n] += s * F[:, j, i]
    np.testing.assert_allclose(pic.gather(p, F, x, y), ref, atol=1e-13)


def test_wrap_edge():
    L = 1.0
    x = np.array([-1e-17, 1.0, 2.5, -0.25, 0.999999999])
    w = pic.wrap(x, L)
    assert np.all(w >= 0) and np.all(w < L)
    np.testing.assert_allclose(w[2:], [0.5, 0.75, 0.999999999])


def test_current_at_nodes_and_modes_match_full_deposit():
    """The direct sums used for full-size sampled checks equal the oracle's
    own deposit (at every sampled node) and numpy's rfft2 of it (at every
    sampled mode), including particles near the periodic seam."""
    from oracle import pic as opic
    from paper_2410_18414_amd import workloads
    for degree in (1, 2, 3):
        w = workloads.weibel(nx=16, ny=8, ppc=6, seed=60 + degree, drift=0.1)
        w["x"][:5] = [0.0, 1e-9, w["lx"] - 1e-9, 0.5 * w["lx"], w["lx"] * 0.999]
        p = opic.Params(w["nx"], w["ny"], w["lx"], w["ly"], degree, "bdf", w["dt"], q=w["q"], m=w["m"])
        part = opic.init_particles(p, w["x"], w["y"], w["P"])
        J = opic.deposit_current(p, part["x"], part["y"], part["v"])
        nodes = [(0, 0), (15, 7), (3, 4), (8, 0), (0, 7)]
        got = opic.current_at_nodes(p, part["x"], part["y"], part["v"], nodes, batch=100)
        ref = np.array([J[:, iy, ix] for ix, iy in nodes])
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(J).max()
        modes = [(0, 0), (1, 0), (3, 5), (8, 4), (5, 7)]
        Jh = np.fft.rfft2(J)
        got = opic.current_modes(p, part["x"], part["y"], part["v"], modes, batch=100)
        ref = np.array([Jh[:, ky, kx] for kx, ky in modes])
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(Jh).max()
