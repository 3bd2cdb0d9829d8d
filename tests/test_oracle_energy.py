"""Pin of the oracle's field energy W against a hand-integrated closed form
(CPU only).

W is the adjoint workload's loss: W = (dx dy / 2) sum_mesh (eps0 |E|^2 +
|B|^2 / mu0) with E = -grad phi - dA/dt and B = curl A (Sec. 2.1-2.2; the time
derivative is each stepper's own: the BDF-k difference of Sec. 3.2, the
staggered difference of Sec. 3.1, v_A of the DIRK system of Sec. 3.3).

The history is planted with one Fourier mode, psi = kx x + ky y (neither the
zero nor a Nyquist mode): phi = Phi cos(psi) and every A level
A_l = alpha_l sin(psi), with different amplitudes per level and component.
Then, by hand,
    grad phi = -Phi sin(psi) (kx, ky),
    dA/dt    = beta sin(psi)          (beta from the stepper's difference),
    E        = (Phi kx - beta_x, Phi ky - beta_y, -beta_z) sin(psi),
    B        = (ky a_z, -kx a_z, kx a_y - ky a_x) cos(psi)   (a: A's amplitude),
and the mesh sums of sin^2 and cos^2 over the N nodes are N/2 each, so
    W = (lx ly / 4) [eps0 |E amplitude|^2 + |B amplitude|^2 / mu0].
The amplitudes are chosen so that every term is of the same size: a sign
error in E, a dropped factor, or an index slip in B changes W.
"""

import numpy as np
import pytest
import torch

from oracle import adjoint, diagnostics, pic

NX, NY, LX, LY = 16, 12, 1.6, 1.5
MODE = (3, 2)
DT = 0.05
C_LIGHT, EPS0 = 1.3, 0.8


def _params(scheme, k=2):
    return pic.Params(NX, NY, LX, LY, 3, scheme, DT, c=C_LIGHT, eps0=EPS0,
                      mu0=1.0 / (C_LIGHT ** 2 * EPS0), bdf_order=k)


def _waves():
    kx, ky = 2 * np.pi * MODE[0] / LX, 2 * np.pi * MODE[1] / LY
    X, Y = np.meshgrid(np.arange(NX) * LX / NX, np.arange(NY) * LY / NY)
    psi = kx * X + ky * Y
    return kx, ky, np.cos(psi), np.sin(psi)


def _spec(f):
    # planted input only: the half spectrum of mesh samples
    return np.fft.rfft2(f)


def _closed_form(kx, ky, Phi, beta, a, eps0, mu0):
    E = np.array([Phi * kx - beta[0], Phi * ky - beta[1], -beta[2]])
    B = np.array([ky * a[2], -kx * a[2], kx * a[1] - ky * a[0]])
    return LX * LY / 4.0 * (eps0 * E @ E + B @ B / mu0)


def _bdf_coefficients(k):
    # textbook BDF-k first-derivative coefficients (step dt), from the golden table
    import json
    import os
    from fractions import Fraction
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "bdf_dirk_coefficients.json")))
    return np.array([float(Fraction(v)) for v in gold["bdf_first_derivative_over_dt"][str(k)]])


def _planted_bdf(p, k):
    kx, ky, cs, sn = _waves()
    rng = np.random.default_rng(10 + k)
    Phi = 0.9
    # A^{n-j}, j = 0..2k-1: amplitudes per level and component
    amp = rng.uniform(0.2, 1.2, (2 * k, 3)) * np.array([1.0, -0.7, 0.5])
    hist = pic.cold_history(p)
    hist["phi"] = [_spec(Phi * cs)] + [_spec(0.3 * (j + 1) * cs) for j in range(2 * k - 1)]
    hist["A"] = [np.stack([_spec(amp[j, l] * sn) for l in range(3)]) for j in range(2 * k)]
    a = _bdf_coefficients(k)
    beta = sum(a[j] * amp[j] for j in range(k + 1)) / DT
    return hist, _closed_form(kx, ky, Phi, beta, amp[0], p.eps0, p.mu0)


def _state(p):
    e = np.zeros(0)
    return pic.State(p, e, e, np.zeros((0, 3)))


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_bdf_energy_closed_form(k):
    p = _params("bdf", k)
    hist, W = _planted_bdf(p, k)
    s = _state(p)
    s.hist = hist
    got = diagnostics.residuals(s)["energy"]
    assert abs(got - W) <= 1e-12 * W, (got, W)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_autograd_energy_closed_form(k):
    """The adjoint workload's loss (oracle/adjoint.py) on the same planted history."""
    p = _params("bdf", k)
    hist, W = _planted_bdf(p, k)
    pr = adjoint.Problem(p)
    th = {key: [torch.tensor(v) for v in hist[key]] for key in ("rho", "phi", "A")}
    got = float(adjoint.energy(pr, th))
    assert abs(got - W) <= 1e-12 * W, (got, W)


@pytest.mark.parametrize("scheme", ["cdf2", "cdf2_semi", "cdf2_explicit"])
def test_cdf2_energy_closed_form(scheme):
    """Staggered levels: E^{n+1/2} with the mean potential of the form (the
    implicit and semi-implicit forms average phi^{n+3/2} and phi^{n-1/2}, the
    explicit form takes phi^{n+1/2}), dA/dt = (A^{n+1} - A^n)/dt, and B from
    (A^{n+1} + A^n)/2."""
    p = _params(scheme)
    kx, ky, cs, sn = _waves()
    ph = [0.7, 1.1, -0.4]                       # phi^{n+3/2}, phi^{n+1/2}, phi^{n-1/2}
    a1, a0 = np.array([0.9, -0.5, 0.6]), np.array([0.3, 0.8, -0.2])   # A^{n+1}, A^n
    hist = pic.cold_history(p)
    hist["phi"] = [_spec(v * cs) for v in ph]
    hist["A"] = [np.stack([_spec(v * sn) for v in a1]), np.stack([_spec(v * sn) for v in a0])]
    Phi = ph[1] if scheme == "cdf2_explicit" else 0.5 * (ph[0] + ph[2])
    W = _closed_form(kx, ky, Phi, (a1 - a0) / DT, 0.5 * (a1 + a0), p.eps0, p.mu0)
    s = _state(p)
    s.hist = hist
    got = diagnostics.residuals(s)["energy"]
    assert abs(got - W) <= 1e-12 * W, (got, W)


@pytest.mark.parametrize("scheme", ["dirk2", "dirk3"])
def test_dirk_energy_closed_form(scheme):
    """The DIRK first-order system carries v_A = dA/dt: E = -grad phi - v_A."""
    p = _params(scheme)
    kx, ky, cs, sn = _waves()
    a0, vA = np.array([0.4, -0.9, 0.7]), np.array([11.0, -6.0, 9.0])
    hist = pic.cold_history(p)
    hist["phi"] = [_spec(0.8 * cs), _spec(0.1 * cs)]
    hist["A"] = [np.stack([_spec(v * sn) for v in a0]), np.stack([_spec(0.5 * v * sn) for v in a0])]
    hist["vA"] = np.stack([_spec(v * sn) for v in vA])
    W = _closed_form(kx, ky, 0.8, vA, a0, p.eps0, p.mu0)
    s = _state(p)
    s.hist = hist
    got = diagnostics.residuals(s)["energy"]
    assert abs(got - W) <= 1e-12 * W, (got, W)
