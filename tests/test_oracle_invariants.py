"""Pins of the oracle's whole step against the paper's theorems (CPU only).

* Gauge residual at round-off every step: implicit CDF-2 (Sec. 3.1 theorem),
  BDF-k (Sec. 3.2 theorem), s-stage DIRK (Sec. 3.3 theorem, continuity implies
  gauge), given the cold start's zero initial residuals.
* the semi-implicit and explicit CDF-2 forms (Sec. 3.1 theorems: gauge iff
  continuity), with Gauss's law in each form's own levels;
* the three-stage DIRK (Sec. 3.3 theorem for any s-stage DIRK: continuity
  implies gauge);
* Gauss's law at round-off for CDF-2 and BDF-k (Sec. 3.1 and 3.2 theorems);
  DIRK-2 is not expected to satisfy it (remark closing Sec. 3.3).
* div B = 0 identically; total charge constant (k = 0 mode of continuity).
* IAEM push closed forms (Sec. 4.1).
* A whole step on a 4 x 4 grid equals a brute-force variant (all-pairs deposit
  and gather with Cox-de Boor splines, direct DFT instead of numpy.fft).
"""

import numpy as np
import pytest

from oracle import diagnostics, pic, spectral
from paper_2410_18414_amd import workloads

EPS = np.finfo(float).eps


def _state(scheme, k=2, degree=2, c=1.0, nx=16, ny=16, ppc=4, seed=7):
    w = workloads.cloud(nx=nx, ny=ny, ppc=ppc, seed=seed, drift=0.3, vth=0.05)
    p = pic.Params(w["nx"], w["ny"], w["lx"], w["ly"], degree, scheme, w["dt"] / c,
                   c=c, eps0=1.0, mu0=1.0 / c ** 2, q=w["q"], m=w["m"], bdf_order=k)
    return pic.State(p, w["x"], w["y"], w["P"])


CASES = [("bdf", 1, 2), ("bdf", 2, 3), ("bdf", 3, 2), ("cdf2", 2, 3), ("cdf2_semi", 2, 2),
         ("cdf2_explicit", 2, 3), ("dirk2", 2, 2), ("dirk3", 2, 3), ("bdf", 2, 4), ("cdf2", 2, 5)]


@pytest.mark.parametrize("scheme,k,degree", CASES)
@pytest.mark.parametrize("c", [1.0, 2.0])
def test_gauge_and_gauss(scheme, k, degree, c):
    s = _state(scheme, k, degree, c)
    worst_gauss = 0.0
    for _ in range(25):
        s.step()
        d = diagnostics.residuals(s)
        if d["gauge_scale"] == 0.0:      # sources at the middle level: a quiet first step
            assert d["gauge_l2"] == 0.0 and d["gauss_l2"] == 0.0
            continue
        assert d["gauge_l2"] <= 1e3 * EPS * d["gauge_scale"], d
        assert d["divB_linf"] == 0.0
        assert abs(d["charge"]) <= 1e3 * EPS * d["gauss_scale"]
        worst_gauss = max(worst_gauss, d["gauss_l2"] / d["gauss_scale"])
    if scheme in ("dirk2", "dirk3"):
        assert worst_gauss > 1e-8     # reported, not guaranteed: clearly above round-off
    else:
        assert worst_gauss <= 1e3 * EPS


def test_push_uniform_static_field():
    """A = 0, grad phi uniform and static: P^n = P^0 - n q dt grad phi exactly."""
    p = pic.Params(8, 8, 1.0, 1.0, 2, "bdf", 0.05, q=-2.0, m=3.0)
    rng = np.random.default_rng(1)
    P0 = rng.normal(0, 1.0, (10, 3))
    g = np.zeros((10, 12))
    g[:, 0], g[:, 1] = 0.3, -0.7
    P, v, vp = P0.copy(), pic.velocity(p, P0, np.zeros((10, 3))), None
    vp = v.copy()
    for n in range(1, 21):
        P, vn = pic.push(p, P, v, vp, g)
        vp, v = v, vn
        np.testing.assert_allclose(P[:, 0], P0[:, 0] - n * p.q * p.dt * 0.3, rtol=1e-13)
        np.testing.assert_allclose(P[:, 1], P0[:, 1] + n * p.q * p.dt * 0.7, rtol=1e-13)
        np.testing.assert_array_equal(P[:, 2], P0[:, 2])


def test_push_constant_A_and_speed_limit():
    p = pic.Params(8, 8, 1.0, 1.0, 2, "bdf", 0.05, q=0.5, m=2.0, c=3.0,
                   eps0=1.0, mu0=1.0 / 9.0)
    rng = np.random.default_rng(2)
    P0 = rng.normal(0, 50.0, (100, 3))
    v0 = pic.velocity(p, P0, np.zeros((100, 3)))
    g = np.zeros((100, 12))
    g[:, 2:5] = [0.4, -1.0, 2.0]
    P, v = pic.push(p, P0, v0, v0, g)
    np.testing.assert_array_equal(P, P0)            # no gradients: P unchanged
    u = P0 - p.q * np.array([0.4, -1.0, 2.0])
    gam = np.sqrt(1 + np.sum(u * u, 1) / (p.m * p.c) ** 2)
    np.testing.assert_allclose(v, u / (p.m * gam[:, None]), rtol=1e-14)   # v = u/(m gamma)
    assert np.all(np.sqrt(np.sum(v * v, 1)) < p.c)


def _cdb(m, t):
    def N(k, x):
        if k == 1:
            return np.where((x >= 0) & (x < 1), 1.0, 0.0)
        return (x * N(k - 1, x) + (k - x) * N(k - 1, x - 1)) / (k - 1)
    return N(m + 1, np.asarray(t, float) + (m + 1) / 2.0)


def _brute_weights(p, x, y):
    """W[n, j, i]: spline weight of node (i, j) for particle n, all periodic images."""
    W = np.zeros((x.shape[0], p.ny, p.nx))
    for j in range(p.ny):
        for i in range(p.nx):
            for ix in (-1, 0, 1):
                for iy in (-1, 0, 1):
                    W[:, j, i] += (_cdb(p.degree, (i * p.dx - x - ix * p.lx) / p.dx)
                                   * _cdb(p.degree, (j * p.dy - y - iy * p.ly) / p.dy))
    return W


def _dft(f):
    ny, nx = f.shape
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    out = np.zeros((ny, nx // 2 + 1), complex)
    for ky in range(ny):
        for kx in range(nx // 2 + 1):
            out[ky, kx] = np.sum(f * np.exp(-2j * np.pi * (kx * ii / nx + ky * jj / ny)))
    return out


def _idft(fh, nx, ny):
    full = np.zeros((ny, nx), complex)
    full[:, : nx // 2 + 1] = fh
    for kx in range(nx // 2 + 1, nx):
        full[:, kx] = np.conj(fh[(-np.arange(ny)) % ny, nx - kx])
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    out = np.zeros((ny, nx))
    for ky in range(ny):
        for kx in range(nx):
            out += (full[ky, kx] * np.exp(2j * np.pi * (kx * ii / nx + ky * jj / ny))).real
    return out / (nx * ny)


@pytest.mark.parametrize("scheme,nx,ny", [("bdf", 4, 4), ("cdf2", 4, 4), ("dirk2", 4, 4),
                                          ("bdf", 5, 3), ("dirk2", 6, 5)])
def test_whole_step_brute_force(scheme, nx, ny):
    rng = np.random.default_rng(5)
    p = pic.Params(nx, ny, 1.0, 1.0, 2, scheme, 0.1, q=-0.4, m=0.5, bdf_order=2)
    x, y = rng.uniform(0, 1, 3), rng.uniform(0, 1, 3)
    P = rng.normal(0, 0.3, (3, 3))
    fast = pic.State(p, x, y, P)
    slow = pic.State(p, x, y, P)
    for _ in range(3):
        fast.step()
        # brute-force variant of the same step
        pt = slow.part
        pt["x"], pt["y"] = pic.position_update(p, pt["x"], pt["y"], pt["v"])
        W = _brute_weights(p, pt["x"], pt["y"])
        J = np.einsum("njl,nc->cjl", W, p.q * pt["v"]) / (p.dx * p.dy)
        Jh = np.stack([_dft(J[c]) for c in range(3)])
        slow.hist, phi_t, A_new = pic.field_update(p, slow.hist, Jh)
        spec = [p.ikx * phi_t, p.iky * phi_t, A_new[0], A_new[1], A_new[2],
                p.ikx * A_new[0], p.ikx * A_new[1], p.ikx * A_new[2],
                p.iky * A_new[0], p.iky * A_new[1], p.iky * A_new[2], phi_t]
        F = np.stack([_idft(f, p.nx, p.ny) for f in spec])
        g = np.einsum("njl,fjl->nf", W, F)
        Pn, vn = pic.push(p, pt["P"], pt["v"], pt["vprev"], g)
        pt["P"], pt["vprev"], pt["v"] = Pn, pt["v"], vn
    for key in ("x", "y", "P", "v", "vprev"):
        np.testing.assert_allclose(fast.part[key], slow.part[key], rtol=0, atol=1e-13)
    np.testing.assert_allclose(fast.fields, F, atol=1e-12)


@pytest.mark.parametrize("scheme,nx,ny", [("bdf", 24, 18), ("cdf2", 21, 15), ("dirk2", 20, 27),
                                          ("bdf", 37, 29)])
def test_gauge_and_gauss_on_other_grids(scheme, nx, ny):
    """Sides that are not powers of two (even, odd, prime): the gauge residual
    (and Gauss's law for BDF-k and CDF-2) at round-off."""
    from paper_2410_18414_amd import workloads
    w = workloads.cloud(nx=nx, ny=ny, ppc=3, seed=nx * ny, drift=0.2, vth=0.05)
    p = pic.Params(w["nx"], w["ny"], w["lx"], w["ly"], 3, scheme, w["dt"], q=w["q"], m=w["m"])
    s = pic.State(p, w["x"], w["y"], w["P"])
    s.step(10)
    r = diagnostics.residuals(s)
    assert r["gauge_l2"] <= 1e3 * EPS * r["gauge_scale"], r
    if scheme != "dirk2":
        assert r["gauss_l2"] <= 1e3 * EPS * r["gauss_scale"], r


@pytest.mark.parametrize("s", [2, 3])
@pytest.mark.parametrize("substep", [False, True])
def test_gauge_with_general_dirk_tableau(s, substep):
    """The Sec. 3.3 theorem for an s-stage DIRK that is not a composition of
    implicit-midpoint steps (Alexander's L-stable tableaux): the gauge
    residual stays at round-off every step, with interpolated and with
    sub-stepped stage currents; charge is conserved."""
    from test_oracle_fields import sdirk
    w = workloads.cloud(nx=16, ny=16, ppc=4, seed=71, drift=0.3, vth=0.05)
    p = pic.Params(w["nx"], w["ny"], w["lx"], w["ly"], 3, "dirk2" if s == 2 else "dirk3", w["dt"] / 1.5,
                   c=1.5, eps0=1.0, mu0=1.0 / 1.5 ** 2, q=w["q"], m=w["m"], dirk_substep=substep,
                   dirk_tableau=sdirk(s))
    st = pic.State(p, w["x"], w["y"], w["P"])
    for _ in range(20):
        st.step()
        d = diagnostics.residuals(st)
        assert d["gauge_l2"] <= 1e3 * EPS * d["gauge_scale"], d
        assert abs(d["charge"]) <= 1e3 * EPS * d["gauss_scale"]
