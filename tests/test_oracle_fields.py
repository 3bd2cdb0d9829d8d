"""Pins of the oracle's spectral operators and time steppers (CPU only).

* FFT usage and derivative symbols against a direct DFT and trig polynomials.
* BDF coefficients against the values the paper prints and the textbook table
  (tests/golden/bdf_dirk_coefficients.json), plus polynomial exactness.
* Each stepper's update against its closed-form single-Fourier-mode
  dispersion relation, source free, with c != 1.
"""

import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import pic, schemes, spectral

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "bdf_dirk_coefficients.json")))


def direct_dft2(f):
    ny, nx = f.shape
    out = np.zeros((ny, nx // 2 + 1), complex)
    for ky in range(ny):
        for kx in range(nx // 2 + 1):
            s = 0.0
            for j in range(ny):
                for i in range(nx):
                    s += f[j, i] * np.exp(-2j * np.pi * (kx * i / nx + ky * j / ny))
            out[ky, kx] = s
    return out


@pytest.mark.parametrize("nx,ny", [(4, 4), (8, 6), (16, 16), (9, 6), (7, 11), (15, 5), (12, 10)])
def test_fft_matches_direct_dft(nx, ny):
    f = np.random.default_rng(nx * ny).normal(size=(ny, nx))
    np.testing.assert_allclose(spectral.fft2(f), direct_dft2(f), atol=1e-11)
    np.testing.assert_allclose(spectral.ifft2(spectral.fft2(f), nx, ny), f, atol=1e-13)


def test_spectral_derivatives_of_trig_polynomial():
    nx, ny, lx, ly = 16, 8, 2.0, 3.0
    ikx, iky, lap = spectral.symbols(nx, ny, lx, ly)
    X, Y = np.meshgrid(np.arange(nx) * lx / nx, np.arange(ny) * ly / ny)
    ax, ay = 2 * np.pi * 3 / lx, 2 * np.pi * 2 / ly
    f = np.sin(ax * X) * np.cos(ay * Y) + 0.5 * np.cos(2 * np.pi * 7 / lx * X)
    fh = spectral.fft2(f)
    dfx = spectral.ifft2(ikx * fh, nx, ny)
    dfy = spectral.ifft2(iky * fh, nx, ny)
    lf = spectral.ifft2(lap * fh, nx, ny)
    np.testing.assert_allclose(
        dfx, ax * np.cos(ax * X) * np.cos(ay * Y)
        - 0.5 * 2 * np.pi * 7 / lx * np.sin(2 * np.pi * 7 / lx * X), atol=1e-12)
    np.testing.assert_allclose(dfy, -ay * np.sin(ax * X) * np.sin(ay * Y), atol=1e-12)
    np.testing.assert_allclose(
        lf, -(ax ** 2 + ay ** 2) * np.sin(ax * X) * np.cos(ay * Y)
        - 0.5 * (2 * np.pi * 7 / lx) ** 2 * np.cos(2 * np.pi * 7 / lx * X), atol=1e-10)


@pytest.mark.parametrize("nx,ny", [(15, 9), (12, 7), (11, 10)])
def test_spectral_derivatives_on_odd_and_other_grids(nx, ny):
    """Sides that are odd or not powers of two: every resolved mode, up to the
    highest one of an odd side (which has no Nyquist partner), is
    differentiated exactly."""
    lx, ly = 1.7, 0.9
    ikx, iky, lap = spectral.symbols(nx, ny, lx, ly)
    X, Y = np.meshgrid(np.arange(nx) * lx / nx, np.arange(ny) * ly / ny)
    mx = (nx - 1) // 2          # highest x mode below any Nyquist index
    my = (ny - 1) // 2
    ax, ay = 2 * np.pi * mx / lx, 2 * np.pi * my / ly
    f = np.cos(ax * X + 0.3) * np.sin(ay * Y - 0.2) + np.sin(2 * np.pi / lx * X)
    fh = spectral.fft2(f)
    dfx = spectral.ifft2(ikx * fh, nx, ny)
    dfy = spectral.ifft2(iky * fh, nx, ny)
    lf = spectral.ifft2(lap * fh, nx, ny)
    np.testing.assert_allclose(dfx, -ax * np.sin(ax * X + 0.3) * np.sin(ay * Y - 0.2)
                               + 2 * np.pi / lx * np.cos(2 * np.pi / lx * X), atol=1e-11)
    np.testing.assert_allclose(dfy, ay * np.cos(ax * X + 0.3) * np.cos(ay * Y - 0.2), atol=1e-11)
    np.testing.assert_allclose(lf, -(ax ** 2 + ay ** 2) * np.cos(ax * X + 0.3) * np.sin(ay * Y - 0.2)
                               - (2 * np.pi / lx) ** 2 * np.sin(2 * np.pi / lx * X), atol=1e-9)
    if nx % 2:
        assert np.count_nonzero(ikx[0] == 0) == 1     # no Nyquist index: only kx = 0 vanishes


def test_nyquist_rule_div_grad_equals_laplacian():
    nx, ny = 8, 8
    ikx, iky, lap = spectral.symbols(nx, ny, 1.0, 1.0)
    np.testing.assert_allclose(ikx * ikx + iky * iky, lap, atol=0)
    # the Nyquist cosine has no derivative under the reading
    X, _ = np.meshgrid(np.arange(nx) / nx, np.arange(ny) / ny)
    fh = spectral.fft2(np.cos(np.pi * nx * X))
    assert np.abs(spectral.ifft2(ikx * fh, nx, ny)).max() < 1e-14


def _frac(s):
    return [Fraction(v) for v in s]


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_bdf_coefficients_golden(k):
    assert schemes.bdf_a_exact(k) == _frac(GOLD["bdf_first_derivative_over_dt"][str(k)])


def test_bdf2_values_printed_in_paper():
    a = schemes.bdf_a_exact(2)
    C = schemes.bdf_C_exact(2)
    assert [v / a[0] for v in a] == _frac(GOLD["bdf2_first_derivative_over_two_thirds_dt"])
    assert [v / C[0] for v in C] == _frac(
        GOLD["bdf2_second_derivative_over_two_thirds_dt_squared"])


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_bdf_polynomial_exactness(k):
    """a reproduces d/dt and C = a*a reproduces d2/dt2 for polynomials of degree <= k."""
    a = schemes.bdf_a_exact(k)
    C = schemes.bdf_C_exact(k)
    n = 11
    for deg in range(k + 1):
        d1 = sum(a[j] * Fraction(n - j) ** deg for j in range(k + 1))
        assert d1 == (deg * Fraction(n) ** (deg - 1) if deg else 0)
        d2 = sum(C[j] * Fraction(n - j) ** deg for j in range(2 * k + 1))
        assert d2 == (deg * (deg - 1) * Fraction(n) ** (deg - 2) if deg >= 2 else 0)


def test_table1_structure():
    """Table 1: C_{2k} = a_k^2, C_{2k-1} = 2 a_{k-1} a_k, C_0 = a_0^2, symmetric sums."""
    for k in range(1, 7):
        a, C = schemes.bdf_a_exact(k), schemes.bdf_C_exact(k)
        assert C[0] == a[0] * a[0] and C[2 * k] == a[k] * a[k]
        assert C[2 * k - 1] == 2 * a[k - 1] * a[k] and C[1] == 2 * a[0] * a[1]
        assert sum(C) == 0 and sum(a) == 0   # consistency: constants have no derivative


def test_dirk2_tableau_reading():
    g = GOLD["dirk2_qin_zhang"]
    A = np.array([[float(Fraction(v)) for v in r] for r in g["A"]])
    np.testing.assert_array_equal(schemes.DIRK2_A, A)
    np.testing.assert_array_equal(schemes.DIRK2_B, [float(Fraction(v)) for v in g["b"]])
    np.testing.assert_array_equal(schemes.DIRK2_C, [float(Fraction(v)) for v in g["c"]])
    np.testing.assert_allclose(schemes.DIRK2_A.sum(1), schemes.DIRK2_C)   # row sums
    # second order: b.1 = 1, b.c = 1/2; symplectic: b_i a_ij + b_j a_ji = b_i b_j
    b, Am = schemes.DIRK2_B, schemes.DIRK2_A
    assert b.sum() == 1.0 and b @ schemes.DIRK2_C == 0.5
    M = b[:, None] * Am + (b[:, None] * Am).T - np.outer(b, b)
    np.testing.assert_allclose(M, 0, atol=1e-15)
    # the printed tableau is not consistent (row sums 1/2, 3/4 vs c = 1/4, 1/4)
    gp = GOLD["dirk2_printed_garbled"]
    Ap = np.array([[float(Fraction(v)) for v in r] for r in gp["A"]])
    assert not np.allclose(Ap.sum(1), [float(Fraction(v)) for v in gp["c"]])


# ---------------------------------------------------------------------------
# closed-form single-mode dispersion (source free, J = rho = 0), c != 1

C_LIGHT = 2.0
MODE = (2, 3)          # (kx index, ky index) on a 16 x 16 grid of size 1.6 x 1.2


def _params(scheme, k=2, dt=0.07):
    return pic.Params(16, 16, 1.6, 1.2, 3, scheme, dt, c=C_LIGHT, eps0=1.0,
                      mu0=1.0 / C_LIGHT ** 2, bdf_order=k)


def _theta(p):
    kx = 2 * np.pi * MODE[0] / p.lx
    ky = 2 * np.pi * MODE[1] / p.ly
    return p.c * np.hypot(kx, ky) * p.dt


def _mode_field(p, val):
    f = np.zeros(p.spec_shape, complex)
    f[MODE[1], MODE[0]] = val
    return f


def _run(p, hist, nsteps):
    J0 = np.zeros((3,) + p.spec_shape, complex)
    for _ in range(nsteps):
        hist, _, _ = pic.field_update(p, hist, J0)
    return hist


@pytest.mark.parametrize("k", [1, 2])
def test_bdf_dispersion(k):
    p = _params("bdf", k)
    th = _theta(p)
    if k == 1:
        z = 1.0 / (1.0 - 1j * th)            # 1 - 1/z = i theta
    else:
        # 3/2 - 2w + w^2/2 = +-i theta, w = 1/z: take the principal (least damped)
        # root, so that round-off in the other modes cannot swamp z^n
        roots = [1.0 / (2.0 + sg * np.sqrt(1.0 + 2j * s * th))
                 for sg in (1, -1) for s in (1, -1)]
        z = max((r for r in roots if abs(r) <= 1 + 1e-14), key=abs)
    hist = pic.cold_history(p)
    hist["phi"] = [_mode_field(p, z ** (-j)) for j in range(2 * k)]
    hist["A"] = [np.stack([_mode_field(p, 0.5 * z ** (-j))] * 3) for j in range(2 * k)]
    n = 100
    out = _run(p, hist, n)
    np.testing.assert_allclose(out["phi"][0][MODE[1], MODE[0]], z ** n, rtol=1e-11)
    np.testing.assert_allclose(out["A"][0][2][MODE[1], MODE[0]], 0.5 * z ** n, rtol=1e-11)


def _bdf_golden(k):
    return [float(Fraction(v)) for v in GOLD["bdf_first_derivative_over_dt"][str(k)]]


def _bdf_roots(k, th):
    """Source free, u^n = z^n solves the BDF-k wave update when the BDF-k
    first-derivative polynomial A(w) = sum_j a_j w^j at w = 1/z equals
    +-i theta, since the second difference is the first applied twice
    (C = a * a, Table 1): A(w)^2 + theta^2 = 0.  The 2k roots z = 1/w from
    numpy.roots of the degree-k polynomials A(w) -+ i theta, with the
    textbook a_j (golden table)."""
    a = _bdf_golden(k)
    zs = []
    for s in (1, -1):
        c = list(reversed(a))
        c[-1] = a[0] - s * 1j * th
        zs += [1.0 / w for w in np.roots(c)]
    return zs


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("dt", [0.02, 0.05])
def test_bdf_k_dispersion_roots(k, dt):
    """Every BDF order against its characteristic roots: the history seeded
    with the dominant eigen-solution z^{-j} comes back as z^n after 100 steps
    (the dominant root, so that round-off in the other eigen-directions cannot
    grow faster than it)."""
    p = _params("bdf", k, dt=dt)
    th = _theta(p)
    z = max(_bdf_roots(k, th), key=abs)
    hist = pic.cold_history(p)
    hist["phi"] = [_mode_field(p, z ** (-j)) for j in range(2 * k)]
    hist["A"] = [np.stack([_mode_field(p, (0.5 - 0.25j) * z ** (-j))] * 3) for j in range(2 * k)]
    n = 100
    out = _run(p, hist, n)
    np.testing.assert_allclose(out["phi"][0][MODE[1], MODE[0]], z ** n, rtol=1e-10)
    np.testing.assert_allclose(out["A"][0][1][MODE[1], MODE[0]], (0.5 - 0.25j) * z ** n, rtol=1e-10)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_bdf_k_stability_on_the_imaginary_axis(k):
    """The remark of Sec. 3.2 that BDF-k beyond k = 2 is only A(alpha)-stable:
    on the wave equation's imaginary eigenvalues, BDF-1 and BDF-2 keep every
    root inside the unit circle, while BDF-3..6 have a range of theta where a
    root leaves it -- and the oracle's update grows by exactly that root."""
    ths = np.linspace(0.05, 6.0, 120)
    worst = max((max(abs(z) for z in _bdf_roots(k, th)), th) for th in ths)
    if k <= 2:
        assert worst[0] <= 1.0
        return
    assert worst[0] > 1.01
    # the oracle at that theta: dt chosen so that c |k| dt = theta for MODE
    p0 = _params("bdf", k)
    p = _params("bdf", k, dt=worst[1] / (_theta(p0) / p0.dt))
    z = max(_bdf_roots(k, _theta(p)), key=abs)
    assert abs(z) > 1.01
    hist = pic.cold_history(p)
    hist["phi"] = [_mode_field(p, z ** (-j)) for j in range(2 * k)]
    out = _run(p, hist, 40)
    np.testing.assert_allclose(out["phi"][0][MODE[1], MODE[0]], z ** 40, rtol=1e-10)


def test_cdf2_dispersion():
    p = _params("cdf2")
    th = _theta(p)
    r = 1.0 / (1.0 + th * th / 2)            # z + 1/z = 2 r, |z| = 1
    z = r + 1j * np.sqrt(1 - r * r)
    hist = pic.cold_history(p)
    hist["phi"] = [_mode_field(p, z ** (-j)) for j in range(3)]
    hist["A"] = [np.stack([_mode_field(p, z ** (-j))] * 3) for j in range(2)]
    n = 100
    out = _run(p, hist, n)
    np.testing.assert_allclose(out["phi"][0][MODE[1], MODE[0]], z ** n, rtol=1e-11)
    np.testing.assert_allclose(out["A"][0][1][MODE[1], MODE[0]], z ** n, rtol=1e-11)
    assert abs(abs(z) - 1) < 1e-15


def test_dirk2_dispersion():
    p = _params("dirk2")
    th = _theta(p)
    om = th / p.dt
    z = ((1 + 0.25j * th) / (1 - 0.25j * th)) ** 2
    hist = pic.cold_history(p)
    hist["phi"] = [_mode_field(p, 1.0), _mode_field(p, 0.0)]
    hist["vphi"] = _mode_field(p, 1j * om)
    hist["A"] = [np.stack([_mode_field(p, 1.0)] * 3), np.zeros((3,) + p.spec_shape, complex)]
    hist["vA"] = np.stack([_mode_field(p, 1j * om)] * 3)
    n = 100
    out = _run(p, hist, n)
    np.testing.assert_allclose(out["phi"][0][MODE[1], MODE[0]], z ** n, rtol=1e-11)
    np.testing.assert_allclose(out["vphi"][MODE[1], MODE[0]], 1j * om * z ** n, rtol=1e-11)
    np.testing.assert_allclose(out["A"][0][0][MODE[1], MODE[0]], z ** n, rtol=1e-11)
    assert abs(abs(z) - 1) < 1e-14


@pytest.mark.parametrize("scheme", ["cdf2_semi", "cdf2_explicit"])
def test_cdf2_other_forms_dispersion(scheme):
    """Source free, the semi-implicit form is the implicit one's recursion,
    L(u^{n+1} + u^{n-1}) = 2 u^n, so z + 1/z = 2/(1 + theta^2/2); the
    explicit form is leapfrog, z + 1/z = 2 - theta^2 (|z| = 1 for theta <= 2,
    the CFL bound of the explicit wave update)."""
    p = _params(scheme, dt=0.05)
    th = _theta(p)
    assert th < 2.0
    r = 1.0 / (1.0 + th * th / 2) if scheme == "cdf2_semi" else 1.0 - th * th / 2
    z = r + 1j * np.sqrt(1 - r * r)
    hist = pic.cold_history(p)
    hist["phi"] = [_mode_field(p, z ** (-j)) for j in range(3)]
    hist["A"] = [np.stack([_mode_field(p, z ** (-j))] * 3) for j in range(2)]
    n = 100
    out = _run(p, hist, n)
    np.testing.assert_allclose(out["phi"][0][MODE[1], MODE[0]], z ** n, rtol=1e-11)
    np.testing.assert_allclose(out["A"][0][2][MODE[1], MODE[0]], z ** n, rtol=1e-11)
    assert abs(abs(z) - 1) < 1e-15


def test_cdf2_explicit_is_unstable_beyond_cfl():
    """Above theta = 2 the leapfrog roots leave the unit circle: a single mode
    grows like the larger root |z| = |r| + sqrt(r^2 - 1), r = 1 - theta^2/2."""
    p = _params("cdf2_explicit", dt=0.09)
    th = _theta(p)
    r = 1.0 - th * th / 2
    assert r < -1.0
    z = r - np.sqrt(r * r - 1)                       # |z| > 1
    hist = pic.cold_history(p)
    hist["phi"] = [_mode_field(p, z ** (-j)) for j in range(3)]
    hist["A"] = [np.stack([_mode_field(p, z ** (-j))] * 3) for j in range(2)]
    out = _run(p, hist, 20)
    np.testing.assert_allclose(out["phi"][0][MODE[1], MODE[0]], z ** 20, rtol=1e-9)


def test_dirk_composition_tableaux():
    """The composition of implicit-midpoint substeps reproduces the Qin-Zhang
    tableau for b = (1/2, 1/2); the three-stage triple-jump composition has
    order four (stability function vs exp, a Taylor check) and modulus one on
    the imaginary axis, and satisfies the symplecticity condition
    b_i a_ij + b_j a_ji - b_i b_j = 0."""
    A, b, c = schemes.dirk_composed([0.5, 0.5])
    np.testing.assert_array_equal(A, schemes.DIRK2_A)
    np.testing.assert_array_equal(c, schemes.DIRK2_C)
    A3, b3, c3 = schemes.DIRK3_A, schemes.DIRK3_B, schemes.DIRK3_C
    assert abs(b3.sum() - 1.0) < 1e-15
    M = b3[:, None] * A3 + (b3[:, None] * A3).T - np.outer(b3, b3)
    np.testing.assert_allclose(M, 0, atol=1e-14)

    def R(z):   # R(z) = 1 + z b^T (I - z A)^{-1} 1
        return 1.0 + z * b3 @ np.linalg.solve(np.eye(3) - z * A3, np.ones(3))
    for th in (0.3, 1.0, 3.0):
        assert abs(abs(R(1j * th)) - 1.0) < 1e-13
    # order 4: the error of R against exp scales as z^5
    e1, e2 = abs(R(0.02) - np.exp(0.02)), abs(R(0.01) - np.exp(0.01))
    assert 25.0 < e1 / e2 < 40.0        # 2^5 = 32


def test_dirk3_dispersion():
    p = _params("dirk3")
    th = _theta(p)
    om = th / p.dt
    z = np.prod([(1 + 0.5j * bi * th) / (1 - 0.5j * bi * th) for bi in schemes.DIRK3_B])
    hist = pic.cold_history(p)
    hist["phi"] = [_mode_field(p, 1.0), _mode_field(p, 0.0)]
    hist["vphi"] = _mode_field(p, 1j * om)
    hist["A"] = [np.stack([_mode_field(p, 1.0)] * 3), np.zeros((3,) + p.spec_shape, complex)]
    hist["vA"] = np.stack([_mode_field(p, 1j * om)] * 3)
    n = 100
    out = _run(p, hist, n)
    np.testing.assert_allclose(out["phi"][0][MODE[1], MODE[0]], z ** n, rtol=1e-10)
    np.testing.assert_allclose(out["vphi"][MODE[1], MODE[0]], 1j * om * z ** n, rtol=1e-10)
    np.testing.assert_allclose(out["A"][0][0][MODE[1], MODE[0]], z ** n, rtol=1e-10)
    assert abs(abs(z) - 1) < 1e-14


# ---------------------------------------------------------------------------
# general s-stage DIRK tableaux (Sec. 3.3 states the method for any tableau)

def sdirk(s):
    """Alexander's singly diagonally implicit tableau of `s` stages from the
    golden expressions (gamma: 1 - 1/sqrt(2), or the root in (1/6, 1/2) of
    6 g^3 - 18 g^2 + 9 g - 1)."""
    if s == 2:
        g = 1.0 - 1.0 / np.sqrt(2.0)
    else:
        r = np.roots([6.0, -18.0, 9.0, -1.0])
        g = float(next(x.real for x in r if abs(x.imag) < 1e-12 and 1 / 6 < x.real < 0.5))
    ev = lambda e: float(eval(e, {"g": g}))  # noqa: E731  (arithmetic of g only)
    t = GOLD["sdirk_alexander"][str(s)]
    return (np.array([[ev(e) for e in row] for row in t["A"]]), np.array([ev(e) for e in t["b"]]),
            np.array([ev(e) for e in t["c"]]))


def _R(A, b, z):
    """Stability function R(z) = 1 + z b^T (I - z A)^{-1} 1."""
    return 1.0 + z * b @ np.linalg.solve(np.eye(len(b)) - z * A, np.ones(len(b)))


@pytest.mark.parametrize("s", [2, 3])
def test_sdirk_tableaux_order_and_stability(s):
    """The golden tableaux are what they claim: consistent (c = row sums),
    of order s (order conditions up to s), L-stable (R -> 0 at -infinity,
    |R| <= 1 on the imaginary axis) -- and, unlike the symplectic
    compositions, dissipative (|R(i theta)| < 1)."""
    A, b, c = sdirk(s)
    np.testing.assert_allclose(A.sum(1), c, atol=1e-15)
    assert abs(b.sum() - 1) < 1e-15 and abs(b @ c - 0.5) < 1e-15
    if s == 3:
        assert abs(b @ c ** 2 - 1 / 3) < 1e-14 and abs(b @ A @ c - 1 / 6) < 1e-14
    assert abs(_R(A, b, -1e9)) < 1e-6
    for th in (0.1, 1.0, 3.0):
        assert abs(_R(A, b, 1j * th)) < 1.0


@pytest.mark.parametrize("s", [2, 3])
def test_general_dirk_dispersion(s):
    """The oracle with a non-composed tableau: the eigen-solution (u, v) =
    (1, i omega) of the source-free wave equation, omega = c |k|, returns
    R(i theta)^n after 100 steps, R from the matrix form of the stability
    function (not the oracle's stage-by-stage recursion)."""
    A, b, c = sdirk(s)
    p = pic.Params(16, 16, 1.6, 1.2, 3, "dirk2" if s == 2 else "dirk3", 0.07, c=C_LIGHT, eps0=1.0,
                   mu0=1.0 / C_LIGHT ** 2, dirk_tableau=(A, b, c))
    th = _theta(p)
    om = th / p.dt
    z = _R(A, b, 1j * th)
    hist = pic.cold_history(p)
    hist["phi"] = [_mode_field(p, 1.0), _mode_field(p, 0.0)]
    hist["vphi"] = _mode_field(p, 1j * om)
    hist["A"] = [np.stack([_mode_field(p, 1.0)] * 3), np.zeros((3,) + p.spec_shape, complex)]
    hist["vA"] = np.stack([_mode_field(p, 1j * om)] * 3)
    n = 100
    out = _run(p, hist, n)
    np.testing.assert_allclose(out["phi"][0][MODE[1], MODE[0]], z ** n, rtol=1e-10)
    np.testing.assert_allclose(out["vphi"][MODE[1], MODE[0]], 1j * om * z ** n, rtol=1e-10)
    np.testing.assert_allclose(out["A"][0][2][MODE[1], MODE[0]], z ** n, rtol=1e-10)
    assert abs(z) < 1.0
