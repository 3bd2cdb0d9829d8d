"""Residual diagnostics of the oracle state (test infrastructure only).

Gauge residual epsilon_1 and Gauss residual per stepper, at the newest level
held in the history after a step:
  BDF-k  (Sec. 3.2): eps1^n = (1/(c^2 dt)) sum_j a_j phi^{n-j} + div A^n;
         E^n = -grad phi^n - (1/dt) sum_j a_j A^{n-j};  Gauss: div E^n - rho^n/eps0.
  CDF-2  (Sec. 3.1): eps1^{n+1} = (phi^{n+3/2} - phi^{n+1/2})/(c^2 dt) + div A^{n+1};
         E^{n+1/2} = -grad (phi^{n+3/2} + phi^{n-1/2})/2 - (A^{n+1} - A^n)/dt;
         Gauss: div E^{n+1/2} - (rho^{n+3/2} + rho^{n-1/2})/(2 eps0).
         Reading for the semi-implicit and explicit forms (the paper states the
         Gauss theorem for the implicit form only; the same steps give): the
         source level rho^{n+1/2}, and for the explicit form the Laplacian's
         level, E^{n+1/2} = -grad phi^{n+1/2} - (A^{n+1} - A^n)/dt.
  DIRK-2 (Sec. 3.3): eps1^{n+1} = -phi^{n+1} + phi^n
         - c^2 h (R^{s,n} div A^n + R^{s,n+1} div A^{n+1}), R = sum b_i (1-c_i), sum b_i c_i.
         Reading: Gauss is reported (not guaranteed, remark closing Sec. 3.3) with
         E^{n+1} = -grad phi^{n+1} - v_A^{n+1}.
         Sub-stepped stage currents (Params.dirk_substep): the gauge is the
         stage-value form, eps1^{n+1} = v_phi^{n+1} + c^2 div A^{n+1} (zero at
         every stage implies the printed phi^{n+1} = phi^n - c^2 h sum b_i div A^(i)
         with A^(i) the RK stage values); Gauss as above.
Norms (the paper does not define them): discrete L2 = sqrt(dx dy sum f^2) and
L-infinity over the mesh.  Field energy W = (dx dy / 2) sum (eps0 |E|^2 + |B|^2/mu0)
with B = curl A (B_x = d_y A_z, B_y = -d_x A_z, B_z = d_x A_y - d_y A_x).
"""

import numpy as np

from . import schemes, spectral


def _real(p, fh):
    return spectral.ifft2(fh, p.nx, p.ny)


def _l2(p, f):
    return float(np.sqrt(p.dx * p.dy * np.sum(f * f)))


def residuals(state):
    p, h = state.p, state.hist
    ikx, iky, lap = p.ikx, p.iky, p.lap
    divA = lambda Ah: ikx * Ah[0] + iky * Ah[1]  # noqa: E731
    if p.scheme == "bdf":
        k = p.bdf_order
        a = schemes.bdf_a(k)
        dphi = sum(a[j] * h["phi"][j] for j in range(k + 1)) / (p.c ** 2 * p.dt)
        dA = sum(a[j] * h["A"][j] for j in range(k + 1)) / p.dt
        gauge_t, gauge_d = dphi, divA(h["A"][0])
        phi, rho = h["phi"][0], h["rho"][0]
        Eh = np.stack([-ikx * phi - dA[0], -iky * phi - dA[1], -dA[2]])
        Ah = h["A"][0]
    elif p.scheme in ("cdf2", "cdf2_semi", "cdf2_explicit"):
        gauge_t = (h["phi"][0] - h["phi"][1]) / (p.c ** 2 * p.dt)
        gauge_d = divA(h["A"][0])
        if p.scheme == "cdf2":
            phim = 0.5 * (h["phi"][0] + h["phi"][2])
            rho = 0.5 * (h["rho"][0] + h["rho"][2])
        elif p.scheme == "cdf2_semi":
            phim = 0.5 * (h["phi"][0] + h["phi"][2])
            rho = h["rho"][1]
        else:
            phim = h["phi"][1]
            rho = h["rho"][1]
        dA = (h["A"][0] - h["A"][1]) / p.dt
        Eh = np.stack([-ikx * phim - dA[0], -iky * phim - dA[1], -dA[2]])
        Ah = 0.5 * (h["A"][0] + h["A"][1])
    else:
        _, b, cc = p.tableau()
        Rn, Rn1 = float(np.sum(b * (1 - cc))), float(np.sum(b * cc))
        if p.dirk_substep:
            # stage-value gauge: v_phi + c^2 div A at the new level
            gauge_t = h["vphi"]
            gauge_d = p.c ** 2 * divA(h["A"][0])
        else:
            gauge_t = -(h["phi"][0] - h["phi"][1])
            gauge_d = -p.c ** 2 * p.dt * (Rn * divA(h["A"][1]) + Rn1 * divA(h["A"][0]))
        phi, rho = h["phi"][0], h["rho"][0]
        Eh = np.stack([-ikx * phi - h["vA"][0], -iky * phi - h["vA"][1], -h["vA"][2]])
        Ah = h["A"][0]
    gauge = _real(p, gauge_t + gauge_d)
    gscale = _l2(p, _real(p, gauge_t)) + _l2(p, _real(p, gauge_d))
    divE = _real(p, ikx * Eh[0] + iky * Eh[1])
    rho_r = _real(p, rho) / p.eps0
    gauss = divE - rho_r
    E = np.stack([_real(p, Eh[i]) for i in range(3)])
    B = np.stack([_real(p, iky * Ah[2]), _real(p, -ikx * Ah[2]),
                  _real(p, ikx * Ah[1] - iky * Ah[0])])
    divB = _real(p, ikx * (iky * Ah[2]) + iky * (-ikx * Ah[2]))
    W = 0.5 * p.dx * p.dy * float(np.sum(p.eps0 * E * E + B * B / p.mu0))
    return dict(gauge_l2=_l2(p, gauge), gauge_linf=float(np.abs(gauge).max()),
                gauge_scale=gscale,
                gauss_l2=_l2(p, gauss), gauss_linf=float(np.abs(gauss).max()),
                gauss_scale=_l2(p, rho_r) + _l2(p, divE),
                charge=float(np.sum(_real(p, h["rho"][0]))) * p.dx * p.dy,
                divB_linf=float(np.abs(divB).max()), energy=W)
