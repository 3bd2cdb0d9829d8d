"""Planted mistakes in the oracle must make its pins fail (CPU only).

Each case patches one plausible error into the oracle (a flipped sign, a
dropped factor, a transposed operand, a wrong coefficient) and re-runs the pin
that should catch it.
"""

import numpy as np
import pytest

from oracle import adjoint, bspline, pic, schemes, spectral
import test_oracle_dirk_substep as D
import test_oracle_energy as E
import test_oracle_fields as F
import test_oracle_invariants as I
import test_oracle_spline_deposit as S


def test_flipped_continuity_sign_breaks_gauge(monkeypatch):
    orig = pic.div
    monkeypatch.setattr(pic, "div", lambda p, V: -orig(p, V))
    with pytest.raises(AssertionError):
        I.test_gauge_and_gauss("bdf", 2, 3, 1.0)


def test_dropped_cell_area_breaks_total_current(monkeypatch):
    orig = pic.deposit_current
    monkeypatch.setattr(pic, "deposit_current",
                        lambda p, x, y, v: orig(p, x, y, v) * p.dx * p.dy)
    with pytest.raises(AssertionError):
        S.test_deposit_total_current()


def test_transposed_gather_breaks_linear_reproduction(monkeypatch):
    orig = pic.gather
    monkeypatch.setattr(pic, "gather", lambda p, f, x, y: orig(p, f, y * p.lx / p.ly,
                                                               x * p.ly / p.lx))
    with pytest.raises(AssertionError):
        S.test_gather_reproduces_linear_fields(3)


def test_wrong_spline_piece_breaks_cox_de_boor(monkeypatch):
    orig = bspline.M
    monkeypatch.setattr(bspline, "M", lambda m, t: orig(m, t) * (1 + 1e-3 * (np.abs(t) > 1)))
    with pytest.raises(AssertionError):
        S.test_spline_matches_cox_de_boor(3)


def test_printed_dirk2_tableau_fails_dispersion(monkeypatch):
    monkeypatch.setattr(schemes, "DIRK2_A", np.array([[0.5, 0.0], [0.25, 0.5]]))
    monkeypatch.setattr(schemes, "DIRK2_C", np.array([0.25, 0.25]))
    with pytest.raises(AssertionError):
        F.test_dirk2_dispersion()


def test_wrong_bdf_alpha_fails_dispersion(monkeypatch):
    orig = schemes.bdf_a
    # a_0 scaled alone: alpha = a_0/(c dt) and the continuity divisor change
    monkeypatch.setattr(schemes, "bdf_a", lambda k: orig(k) * np.r_[1.1, np.ones(k)])
    with pytest.raises(AssertionError):
        F.test_bdf_dispersion(2)


def test_missing_c2_in_dirk_kv_fails_dispersion(monkeypatch):
    """The c^2 the specialised DIRK stage equations drop is caught with c != 1."""
    src = pic._dirk_update

    def patched(p, hist, Jh):
        # the same update with k^v's source term lacking c^2, i.e. c2 -> 1 there
        A_t, b, cc = schemes.DIRK2_A, schemes.DIRK2_B, schemes.DIRK2_C
        h, c2, lap = p.dt, p.c ** 2, p.lap

        def advance(u, v, Sv):
            ku, kv = [], []
            for i in range(2):
                U = u + h * sum(A_t[i, j] * ku[j] for j in range(i))
                V = v + h * sum(A_t[i, j] * kv[j] for j in range(i))
                Li = 1.0 - (h * A_t[i, i] * p.c) ** 2 * lap
                ku.append((V + h * A_t[i, i] * c2 * (Sv[i] + lap * U)) / Li)
                kv.append(((Sv[i] + lap * U) + h * A_t[i, i] * c2 * lap * V) / Li)
            return (u + h * sum(b[i] * ku[i] for i in range(2)),
                    v + h * sum(b[i] * kv[i] for i in range(2)))
        z = [np.zeros(p.spec_shape)] * 2
        phi, vphi = advance(hist["phi"][0], hist["vphi"], z)
        A = np.empty_like(Jh)
        vA = np.empty_like(Jh)
        for l in range(3):
            A[l], vA[l] = advance(hist["A"][0][l], hist["vA"][l], z)
        return (dict(rho=hist["rho"], phi=[phi, hist["phi"][0]], vphi=vphi,
                     A=[A, hist["A"][0]], vA=vA, J=Jh), phi, A)
    assert src is not None
    monkeypatch.setattr(pic, "_dirk_update", patched)
    with pytest.raises(AssertionError):
        F.test_dirk2_dispersion()


def test_linear_stage_rho_with_substepped_currents_breaks_gauge(monkeypatch):
    """The stage charge densities interpolated linearly between rho^n and
    rho^{n+1} (Sec. 3.3's interpolation) while the currents are sub-stepped."""
    def linear(A_t, b, cc, rho_n, dv, h):
        rho_new = rho_n - h * sum(b[i] * dv[i] for i in range(len(b)))
        return [(1 - cc[i]) * rho_n + cc[i] * rho_new for i in range(len(b))]
    monkeypatch.setattr(pic, "_stage_rho", linear)
    with pytest.raises(AssertionError):
        D.test_gauge_and_gauss_at_round_off("dirk2")


def test_wrong_bdf4_coefficient_fails_dispersion(monkeypatch):
    """A sign slip in one term of the backward-difference series (BDF-4's
    a_3) moves the characteristic roots."""
    orig = schemes.bdf_a

    def patched(k):
        a = orig(k)
        if k == 4:
            a = a.copy()
            a[3] = -a[3]
        return a
    monkeypatch.setattr(schemes, "bdf_a", patched)
    with pytest.raises(AssertionError):
        F.test_bdf_k_dispersion_roots(4, 0.02)


def test_flipped_time_derivative_in_E_fails_energy(monkeypatch):
    """E = -grad phi + dA/dt (the sign of the time-derivative term flipped)."""
    orig = schemes.bdf_a
    monkeypatch.setattr(schemes, "bdf_a", lambda k: -orig(k))
    with pytest.raises(AssertionError):
        E.test_bdf_energy_closed_form(2)


def test_transposed_derivatives_fail_energy(monkeypatch):
    """d/dx and d/dy symbols exchanged (a transposed operand in grad and curl)."""
    orig = spectral.symbols

    def swapped(nx, ny, lx, ly):
        ikx, iky, lap = orig(nx, ny, lx, ly)
        return iky, ikx, lap
    monkeypatch.setattr(spectral, "symbols", swapped)
    with pytest.raises(AssertionError):
        E.test_cdf2_energy_closed_form("cdf2")


def test_curl_index_slip_fails_energy(monkeypatch):
    """B_z = d_x A_y + d_y A_x (the sign of curl's second term lost) in the
    adjoint workload's loss."""
    import torch

    def patched(pr, hist):
        p = pr.p
        a = pr.a
        phi = hist["phi"][0]
        A0 = hist["A"][0]
        dA = sum(a[j] * hist["A"][j] for j in range(p.bdf_order + 1)) / p.dt
        Eh = [-pr.ikx * phi - dA[0], -pr.iky * phi - dA[1], -dA[2]]
        Bh = [pr.iky * A0[2], -pr.ikx * A0[2], pr.ikx * A0[1] + pr.iky * A0[0]]
        r = lambda f: torch.fft.irfft2(f, s=(p.ny, p.nx))  # noqa: E731
        return 0.5 * p.dx * p.dy * (p.eps0 * sum(r(e) ** 2 for e in Eh) + sum(r(b) ** 2 for b in Bh) / p.mu0).sum()
    monkeypatch.setattr(adjoint, "energy", patched)
    with pytest.raises(AssertionError):
        E.test_autograd_energy_closed_form(2)


def test_ignored_dirk_tableau_fails_dispersion(monkeypatch):
    """A general tableau silently replaced by the scheme's own."""
    monkeypatch.setattr(pic.Params, "tableau", lambda self: schemes.dirk_tableau(self.scheme))
    with pytest.raises(AssertionError):
        F.test_general_dirk_dispersion(2)
