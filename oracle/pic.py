"""Algorithm 1 of arXiv 2410.18414 in plain FP64 (oracle; test infrastructure only).

One PIC step (Algorithm 1, Sec. 4.2), for one mobile species of macro-particles
on a periodic 2-D grid, 2D3V (x, y; three momentum/velocity components):

  1. x^{n+1} = x^n + v^n dt, wrapped into [0, L)             (IAEM, Sec. 4.1)
  2. J^{n+1} = sum_p q v_p^n S(x - x_p^{n+1})                 (Sec. 2.2, Sec. 4.1)
  3. rho from the continuity equation, in the stepper's own form
  4. phi, A by BDF-k / implicit CDF-2 / DIRK-2, L^{-1} by FFT  (Sec. 3)
  5. spectral gradients of phi~ and A on the mesh             (Sec. 4.1)
  6. gather at x^{n+1} with the same spline S
  7. v* = 2 v^n - v^{n-1};  P^{n+1} = P^n + q(-grad phi~ + (grad A) . v*) dt;
     v^{n+1} = c^2 (P - qA) / sqrt(c^2 (P - qA)^2 + (m c^2)^2)
  8. shift the history

Readings (the paper is silent, ambiguous or misprinted):
  * BDF continuity: Algorithm 1 prints rho^{n+1} with flipped signs and a
    shifted index; the defining equation of Sec. 3.2 (the BDF-k continuity
    equation) is followed: rho^{n+1} = -(1/a_0)[sum_{j>=1} a_j rho^{n+1-j}
    + dt div J^{n+1}].
  * BDF wave equations: "1/(Delta c^2)" is read as 1/c^2; the A source is
    mu0 J (the update formula prints rho/eps0); alpha = a_0/(c dt), the
    Helmholtz solve divides by C_0 = a_0^2; the Laplacian acts on level n+1.
  * DIRK stage equations for k^v: the factor c^2 on the source and on the
    Laplacian of the stage value is restored (it is present in the generic
    stage equations of Sec. 3.3 and dropped in the specialised ones).
  * The DIRK "gauge update" for phi is the gauge constraint, used as the
    diagnostic; phi is advanced by its own stage equations.
  * CDF-2 is the implicit form (sources averaged over n+1 and n-1); the
    semi-implicit ("cdf2_semi": sources rho^{n+1/2}, J^n, Laplacian averaged
    over n+1 and n-1) and explicit ("cdf2_explicit": sources rho^{n+1/2}, J^n,
    Laplacian at n) forms of Sec. 3.1 are the same staggered scheme with the
    other wave updates.  All three keep rho^{n+3/2} from the staggered
    continuity equation with J^{n+1} (given J^{n, n+1}, Sec. 3.1) and use
    phi~ = (phi^{n+3/2} + phi^{n+1/2})/2 for the push.
  * v^{-1} by Taylor expansion: with the cold start below the force at t=0 is
    zero, so v^{-1} = v^0.
  * Cold start: immobile ions are the negative of the t=0 electron charge, so
    rho^0 = 0; every field history level with n <= 0 is zero.
  * A position that wraps to exactly L (floating point) is set to 0.
  * (grad A . v*)_j = sum_l v*_l d_j A_l; d/dz = 0 in 2-D, so P_z is constant.

The naive comparison (Sec. 5.1, the "naive update" of the Weibel figures;
Params(naive=True)): step 3 is replaced by mapping rho^{n+1} to the mesh with
the same spline as J (the PIC charge density of Sec. 2.2), plus the immobile
ion background, which is the negative of the t = 0 electron charge (so
rho^0 = 0 as in the cold start).  Readings: rho is deposited at x^{n+1}, the
positions J^{n+1} is deposited at; BDF-k and DIRK-2 only, since CDF-2 needs
rho at half levels, which the particle positions never occupy.

v* in the current (Params(jvstar=True); Sec. 4.2 allows it as an alternative
to v^n): step 2 becomes J^{n+1} = sum_p q v*_p S(x - x_p^{n+1}) with the push's
extrapolation v* = 2 v^n - v^{n-1}; step 1 still moves the particles with v^n.

DIRK stage currents by particle sub-stepping (Params(dirk_substep=True), the
alternative to linear interpolation named with the DIRK continuity update of
Algorithm 1): stage i deposits J^(i) = sum_p q v_p^n S(x - x_p^n - c_i dt v_p^n),
the particles advanced by the IAEM position update over c_i dt (the same
"position places the weight, v^n carries the value" rule as J^{n+1}).
Reading: the stage charge densities are the Runge-Kutta stage values of the
continuity equation, rho^(i) = rho^n - dt sum_{j<=i} a_ij div J^(j), whose
final stage is the printed rho^{n+1} = rho^n - dt sum_i b_i div J^(i).  (The
linear interpolation between rho^n and rho^{n+1} that Sec. 3.3 uses holds the
gauge only for linearly interpolated currents.)  With this reading the RK
stages keep v_phi + c^2 div A = 0 and Gauss's law with E = -grad phi - v_A
exactly, since the pair of those two residuals obeys a source-free linear
system that the RK method advances from zero.  The J history level holds
sum_i b_i J^(i), the current of the step's continuity update.
"""

import numpy as np

from . import bspline, spectral, schemes

# order of the 12 mesh fields the gather interpolates (slot 11 is phi~ itself)
FIELD_NAMES = ("dphi_dx", "dphi_dy", "Ax", "Ay", "Az",
               "dAx_dx", "dAy_dx", "dAz_dx", "dAx_dy", "dAy_dy", "dAz_dy", "phi")


# the staggered centred-difference schemes of Sec. 3.1
CDF2_FORMS = ("cdf2", "cdf2_semi", "cdf2_explicit")
# the DIRK schemes of Sec. 3.3: the two-stage Qin-Zhang tableau and the
# three-stage fourth-order composition (schemes.dirk_tableau)
DIRK_FORMS = ("dirk2", "dirk3")


class Params:
    def __init__(self, nx, ny, lx, ly, degree, scheme, dt, c=1.0, eps0=1.0,
                 mu0=1.0, q=-1.0, m=1.0, bdf_order=2, naive=False, jvstar=False,
                 dirk_substep=False, dirk_tableau=None):
        if scheme not in ("bdf",) + CDF2_FORMS + DIRK_FORMS:
            raise ValueError(scheme)
        # a general s-stage DIRK tableau (A lower triangular, b, c) replacing
        # the scheme's own (Sec. 3.3 states the method for any tableau)
        if dirk_tableau is not None:
            if scheme not in DIRK_FORMS:
                raise ValueError("a DIRK tableau needs a DIRK scheme")
            A_t, b, cc = (np.array(t, np.float64) for t in dirk_tableau)
            if A_t.shape != (len(b), len(b)) or cc.shape != b.shape or np.any(np.triu(A_t, 1) != 0):
                raise ValueError("the tableau must be a lower-triangular s x s A with b, c of length s")
            self.dirk_tab = (A_t, b, cc)
        else:
            self.dirk_tab = None
        if naive and scheme in CDF2_FORMS:
            raise ValueError("the naive charge deposit needs BDF-k or DIRK-2")
        self.naive = bool(naive)
        self.jvstar = bool(jvstar)
        if dirk_substep and (scheme not in DIRK_FORMS or naive):
            raise ValueError("sub-stepped stage currents need a DIRK scheme and continuity")
        self.dirk_substep = bool(dirk_substep)
        if abs(c * c * eps0 * mu0 - 1.0) > 1e-12:
            raise ValueError("c^2 eps0 mu0 must equal 1")
        self.nx, self.ny, self.lx, self.ly = int(nx), int(ny), float(lx), float(ly)
        self.dx, self.dy = self.lx / self.nx, self.ly / self.ny
        self.degree, self.scheme, self.bdf_order = int(degree), scheme, int(bdf_order)
        self.dt, self.c, self.eps0, self.mu0 = float(dt), float(c), float(eps0), float(mu0)
        self.q, self.m = float(q), float(m)
        self.ikx, self.iky, self.lap = spectral.symbols(self.nx, self.ny, self.lx, self.ly)

    @property
    def spec_shape(self):
        return (self.ny, self.nx // 2 + 1)

    def tableau(self):
        """(A, b, c) of the DIRK stepper: the one given, else the scheme's."""
        return self.dirk_tab if self.dirk_tab is not None else schemes.dirk_tableau(self.scheme)


# ----------------------------------------------------------------------------
# particles

def wrap(x, L):
    x = x - L * np.floor(x / L)
    x = np.where(x >= L, 0.0, x)
    return x


def velocity(p, P, A):
    """v = c^2 (P - qA) / sqrt(c^2 |P - qA|^2 + (m c^2)^2)  (Sec. 2.2)."""
    u = P - p.q * A
    s = np.sqrt(p.c ** 2 * np.sum(u * u, axis=1) + (p.m * p.c ** 2) ** 2)
    return p.c ** 2 * u / s[:, None]


def init_particles(p, x, y, P):
    """Given x^0, P^0 with A^0 = 0: v^0 from P^0, and v^{-1} = v^0 (cold start)."""
    x = wrap(np.asarray(x, np.float64), p.lx)
    y = wrap(np.asarray(y, np.float64), p.ly)
    P = np.array(P, np.float64)
    v = velocity(p, P, np.zeros_like(P))
    return dict(x=x, y=y, P=P, v=v, vprev=v.copy())


def position_update(p, x, y, v):
    return wrap(x + v[:, 0] * p.dt, p.lx), wrap(y + v[:, 1] * p.dt, p.ly)


def stage_positions(p, x, y, v, frac):
    """The IAEM position update over frac * dt (a DIRK stage time)."""
    return wrap(x + v[:, 0] * (frac * p.dt), p.lx), wrap(y + v[:, 1] * (frac * p.dt), p.ly)


def deposit_current(p, x, y, v):
    """J(x_g) = sum_p q v_p S(x_g - x_p), S = M(dx)M(dy)/(dx dy); shape [3, ny, nx]."""
    gx, wx = bspline.stencil(p.degree, x / p.dx)
    gy, wy = bspline.stencil(p.degree, y / p.dy)
    n = p.nx * p.ny
    J = np.zeros((3, n))
    qv = p.q * v
    for a in range(gx.shape[1]):
        for b in range(gy.shape[1]):
            idx = (gy[:, b] % p.ny) * p.nx + (gx[:, a] % p.nx)
            w = wx[:, a] * wy[:, b] / (p.dx * p.dy)
            for c in range(3):
                J[c] += np.bincount(idx, weights=w * qv[:, c], minlength=n)
    return J.reshape(3, p.ny, p.nx)


def deposit_charge(p, x, y):
    """rho(x_g) = sum_p q S(x_g - x_p) (Sec. 2.2, PIC charge density); [ny, nx]."""
    gx, wx = bspline.stencil(p.degree, x / p.dx)
    gy, wy = bspline.stencil(p.degree, y / p.dy)
    n = p.nx * p.ny
    rho = np.zeros(n)
    for a in range(gx.shape[1]):
        for b in range(gy.shape[1]):
            idx = (gy[:, b] % p.ny) * p.nx + (gx[:, a] % p.nx)
            rho += np.bincount(idx, weights=p.q * wx[:, a] * wy[:, b] / (p.dx * p.dy), minlength=n)
    return rho.reshape(p.ny, p.nx)


def current_at_nodes(p, x, y, v, nodes, batch=1 << 23):
    """J at selected mesh nodes straight from the definition
    J(x_g) = sum_p q v_p M(x_g/dx - x_p/dx) M(y_g/dy - y_p/dy) / (dx dy),
    each particle taken at its periodic image nearest the node.  nodes is a
    list of (ix, iy); returns [len(nodes), 3].  For workloads too large for
    deposit_current's per-particle index arrays."""
    out = np.zeros((len(nodes), 3))
    sup = bspline.SUPPORT[p.degree]
    for s in range(0, x.shape[0], batch):
        xi, eta, vb = x[s:s + batch] / p.dx, y[s:s + batch] / p.dy, v[s:s + batch]
        for k, (ix, iy) in enumerate(nodes):
            tx = ix - xi
            tx -= p.nx * np.round(tx / p.nx)
            ty = iy - eta
            ty -= p.ny * np.round(ty / p.ny)
            sel = (np.abs(tx) < sup) & (np.abs(ty) < sup)
            w = bspline.M(p.degree, tx[sel]) * bspline.M(p.degree, ty[sel]) / (p.dx * p.dy)
            out[k] += p.q * (w[:, None] * vb[sel]).sum(axis=0)
    return out


def current_modes(p, x, y, v, modes, batch=1 << 23):
    """rfft2 of J at selected modes (kx, ky) (numpy's unnormalised convention,
    kx in 0..nx/2, ky in 0..ny-1), summed over particles: the DFT of one
    particle's deposit is its weight on each stencil node times the node's
    phase.  Returns [len(modes), 3] complex."""
    out = np.zeros((len(modes), 3), np.complex128)
    for s in range(0, x.shape[0], batch):
        gx, wx = bspline.stencil(p.degree, x[s:s + batch] / p.dx)
        gy, wy = bspline.stencil(p.degree, y[s:s + batch] / p.dy)
        qv = p.q * v[s:s + batch] / (p.dx * p.dy)
        offs = np.arange(gx.shape[1])  # stencil nodes are g[:, 0] + offs
        bx = np.mod(gx[:, 0], p.nx)
        by = np.mod(gy[:, 0], p.ny)
        for k, (kx, ky) in enumerate(modes):
            # sum_a w_a e^{-2 pi i kx (g0 + a)/nx}: the phase of the first node
            # (a table over node indices) times the weights' transform
            cx = np.exp(-2j * np.pi * kx * offs / p.nx)
            cy = np.exp(-2j * np.pi * ky * offs / p.ny)
            tx = np.exp(-2j * np.pi * kx * np.arange(p.nx) / p.nx)
            ty = np.exp(-2j * np.pi * ky * np.arange(p.ny) / p.ny)
            fx = tx[bx] * (wx @ cx.real + 1j * (wx @ cx.imag))
            fy = ty[by] * (wy @ cy.real + 1j * (wy @ cy.imag))
            f = fx * fy
            out[k] += f.real @ qv + 1j * (f.imag @ qv)
    return out


def gather(p, fields, x, y):
    """Interpolate mesh fields [F, ny, nx] at the particles with the same spline."""
    gx, wx = bspline.stencil(p.degree, x / p.dx)
    gy, wy = bspline.stencil(p.degree, y / p.dy)
    F = fields.reshape(fields.shape[0], -1)
    out = np.zeros((x.shape[0], fields.shape[0]))
    for a in range(gx.shape[1]):
        for b in range(gy.shape[1]):
            idx = (gy[:, b] % p.ny) * p.nx + (gx[:, a] % p.nx)
            out += (wx[:, a] * wy[:, b])[:, None] * F[:, idx].T
    return out


def push(p, P, v, vprev, g):
    """IAEM momentum and velocity update (Sec. 4.1) from gathered fields g [N, 12]."""
    vs = 2.0 * v - vprev
    Fx = -g[:, 0] + vs[:, 0] * g[:, 5] + vs[:, 1] * g[:, 6] + vs[:, 2] * g[:, 7]
    Fy = -g[:, 1] + vs[:, 0] * g[:, 8] + vs[:, 1] * g[:, 9] + vs[:, 2] * g[:, 10]
    Pn = P.copy()
    Pn[:, 0] += p.q * Fx * p.dt
    Pn[:, 1] += p.q * Fy * p.dt
    vn = velocity(p, Pn, g[:, 2:5])
    return Pn, vn


# ----------------------------------------------------------------------------
# fields

def cold_history(p):
    """Zero history for the chosen stepper (all levels n <= 0 vanish)."""
    z = lambda: np.zeros(p.spec_shape, np.complex128)  # noqa: E731
    z3 = lambda: np.zeros((3,) + p.spec_shape, np.complex128)  # noqa: E731
    if p.scheme == "bdf":
        k = p.bdf_order
        return dict(rho=[z() for _ in range(k)], phi=[z() for _ in range(2 * k)],
                    A=[z3() for _ in range(2 * k)])
    if p.scheme in CDF2_FORMS:
        return dict(rho=[z() for _ in range(3)], phi=[z() for _ in range(3)],
                    A=[z3() for _ in range(2)], J=[z3() for _ in range(2)])
    return dict(rho=[z(), z()], phi=[z(), z()], vphi=z(), A=[z3(), z3()], vA=z3(), J=z3())


def div(p, Vh):
    return p.ikx * Vh[0] + p.iky * Vh[1]


def field_update(p, hist, Jh, rho_h=None):
    """Continuity + wave update given J^{n+1} (spectral).  Returns (hist', phi~, A).
    rho_h: the deposited rho^{n+1} (spectral) of the naive comparison, used in
    place of continuity (BDF-k and DIRK-2)."""
    if rho_h is not None and p.scheme in CDF2_FORMS:
        raise ValueError("the naive charge deposit needs BDF-k or DIRK-2")
    extra = () if rho_h is None else (rho_h,)
    if p.scheme == "bdf":
        return _bdf_update(p, hist, Jh, *extra)
    if p.scheme == "cdf2":
        return _cdf2_update(p, hist, Jh)
    if p.scheme in CDF2_FORMS:
        return _cdf2_other_update(p, hist, Jh)
    return _dirk_update(p, hist, Jh, *extra)


def _bdf_update(p, hist, Jh, rho_h=None):
    # Sec. 3.2: BDF-k continuity, wave equations and the L^{-1} update form
    k = p.bdf_order
    a = schemes.bdf_a(k)
    C = schemes.bdf_C(k)
    if rho_h is None:
        rho_new = -(sum(a[j] * hist["rho"][j - 1] for j in range(1, k + 1))
                    + p.dt * div(p, Jh)) / a[0]
    else:
        rho_new = rho_h
    alpha2 = (a[0] / (p.c * p.dt)) ** 2
    Lh = 1.0 - p.lap / alpha2
    phi_new = (rho_new / (p.eps0 * alpha2)
               - sum(C[i] / C[0] * hist["phi"][i - 1] for i in range(1, 2 * k + 1))) / Lh
    A_new = (p.mu0 * Jh / alpha2
             - sum(C[i] / C[0] * hist["A"][i - 1] for i in range(1, 2 * k + 1))) / Lh
    out = dict(rho=[rho_new] + hist["rho"][:-1], phi=[phi_new] + hist["phi"][:-1],
               A=[A_new] + hist["A"][:-1])
    return out, phi_new, A_new


def _cdf2_update(p, hist, Jh):
    # Sec. 3.1: staggered continuity and the Crank-Nicolson form L(u^{n+1}+u^{n-1})
    #   = 2u^n + Gamma/alpha^2 with alpha = sqrt(2)/(c dt)
    rho_h, rho_mh = hist["rho"][0], hist["rho"][1]          # rho^{n+1/2}, rho^{n-1/2}
    phi_h, phi_mh = hist["phi"][0], hist["phi"][1]          # phi^{n+1/2}, phi^{n-1/2}
    A_n, A_m = hist["A"][0], hist["A"][1]                   # A^n, A^{n-1}
    J_m = hist["J"][1]                                      # J^{n-1}
    rho_new = rho_h - p.dt * div(p, Jh)                     # rho^{n+3/2}
    alpha2 = 2.0 / (p.c * p.dt) ** 2
    Lh = 1.0 - p.lap / alpha2
    phi_new = -phi_mh + (2.0 * phi_h + (rho_new + rho_mh) / (alpha2 * p.eps0)) / Lh
    A_new = -A_m + (2.0 * A_n + p.mu0 * (Jh + J_m) / alpha2) / Lh
    phi_tilde = 0.5 * (phi_new + phi_h)                     # Sec. 4.1, staggered phi
    out = dict(rho=[rho_new, rho_h, rho_mh], phi=[phi_new, phi_h, phi_mh],
               A=[A_new, A_n], J=[Jh, hist["J"][0]])
    return out, phi_tilde, A_new


def _cdf2_other_update(p, hist, Jh):
    # Sec. 3.1, semi-implicit and explicit forms: the wave equations take the
    # sources at the middle level (rho^{n+1/2}, J^n); the semi-implicit form
    # averages the Laplacian over n+1 and n-1 (the L solve of the implicit
    # form with Gamma = 2 S^n), the explicit form takes it at level n (no solve)
    rho_h, rho_mh = hist["rho"][0], hist["rho"][1]          # rho^{n+1/2}, rho^{n-1/2}
    phi_h, phi_mh = hist["phi"][0], hist["phi"][1]          # phi^{n+1/2}, phi^{n-1/2}
    A_n, A_m = hist["A"][0], hist["A"][1]                   # A^n, A^{n-1}
    J_n = hist["J"][0]                                      # J^n
    rho_new = rho_h - p.dt * div(p, Jh)                     # rho^{n+3/2}, continuity
    if p.scheme == "cdf2_semi":
        alpha2 = 2.0 / (p.c * p.dt) ** 2
        Lh = 1.0 - p.lap / alpha2
        phi_new = -phi_mh + (2.0 * phi_h + 2.0 * rho_h / (alpha2 * p.eps0)) / Lh
        A_new = -A_m + (2.0 * A_n + 2.0 * p.mu0 * J_n / alpha2) / Lh
    else:
        c2dt2 = (p.c * p.dt) ** 2
        phi_new = 2.0 * phi_h - phi_mh + c2dt2 * (p.lap * phi_h + rho_h / p.eps0)
        A_new = 2.0 * A_n - A_m + c2dt2 * (p.lap * A_n + p.mu0 * J_n)
    phi_tilde = 0.5 * (phi_new + phi_h)
    out = dict(rho=[rho_new, rho_h, rho_mh], phi=[phi_new, phi_h, phi_mh],
               A=[A_new, A_n], J=[Jh, J_n])
    return out, phi_tilde, A_new


def _stage_rho(A_t, b, cc, rho_n, dv, h):
    """RK stage values of the continuity equation rho' = -div J given the
    stage divergences dv: rho^(i) = rho^n - h sum_{j<=i} a_ij dv_j."""
    return [rho_n - h * sum(A_t[i, j] * dv[j] for j in range(i + 1)) for i in range(len(b))]


def _dirk_update(p, hist, Jh, rho_h=None):
    # Sec. 3.3: s-stage DIRK on (u, v) with u' = v, v' = c^2 (S + Lap u)
    # Jh: J^{n+1}, or with dirk_substep the s stage currents [s, 3, ...]
    A_t, b, cc = p.tableau()
    s = len(b)
    h, c2, lap = p.dt, p.c ** 2, p.lap
    rho_n = hist["rho"][0]
    if p.dirk_substep:
        J_st = [Jh[i] for i in range(s)]
        dv = [div(p, J_st[i]) for i in range(s)]
        rho_new = rho_n - h * sum(b[i] * dv[i] for i in range(s))
        rho_st = _stage_rho(A_t, b, cc, rho_n, dv, h)
        J_keep = sum(b[i] * J_st[i] for i in range(s))
    else:
        J_n = hist["J"]
        J_st = [(1.0 - cc[i]) * J_n + cc[i] * Jh for i in range(s)]
        if rho_h is None:
            rho_new = rho_n - h * sum(b[i] * div(p, J_st[i]) for i in range(s))
        else:
            rho_new = rho_h
        rho_st = [(1.0 - cc[i]) * rho_n + cc[i] * rho_new for i in range(s)]
        J_keep = Jh

    def advance(u, v, S):
        ku, kv = [], []
        for i in range(s):
            U = u + h * sum(A_t[i, j] * ku[j] for j in range(i))
            V = v + h * sum(A_t[i, j] * kv[j] for j in range(i))
            Li = 1.0 - (h * A_t[i, i] * p.c) ** 2 * lap
            ku.append((V + h * A_t[i, i] * c2 * (S[i] + lap * U)) / Li)
            kv.append((c2 * (S[i] + lap * U) + h * A_t[i, i] * c2 * lap * V) / Li)
        return (u + h * sum(b[i] * ku[i] for i in range(s)),
                v + h * sum(b[i] * kv[i] for i in range(s)))

    phi_new, vphi_new = advance(hist["phi"][0], hist["vphi"],
                                [rho_st[i] / p.eps0 for i in range(s)])
    A_new = np.empty_like(J_keep)
    vA_new = np.empty_like(J_keep)
    for l in range(3):
        A_new[l], vA_new[l] = advance(hist["A"][0][l], hist["vA"][l],
                                      [p.mu0 * J_st[i][l] for i in range(s)])
    out = dict(rho=[rho_new, rho_n], phi=[phi_new, hist["phi"][0]], vphi=vphi_new,
               A=[A_new, hist["A"][0]], vA=vA_new, J=J_keep)
    return out, phi_new, A_new


def gradient_fields(p, phi_h, A_h):
    """The 12 mesh fields (order FIELD_NAMES) by spectral multiply + inverse FFT."""
    spec = [p.ikx * phi_h, p.iky * phi_h, A_h[0], A_h[1], A_h[2],
            p.ikx * A_h[0], p.ikx * A_h[1], p.ikx * A_h[2],
            p.iky * A_h[0], p.iky * A_h[1], p.iky * A_h[2], phi_h]
    return np.stack([spectral.ifft2(f, p.nx, p.ny) for f in spec])


# ----------------------------------------------------------------------------
# the whole step

class State:
    """Particles + field history; `step()` runs Algorithm 1 once."""

    def __init__(self, p, x, y, P):
        self.p = p
        self.part = init_particles(p, x, y, P)
        self.hist = cold_history(p)
        self.J = None
        self.rho = None
        self.fields = None
        self.n = 0
        # naive comparison: immobile ions = minus the t = 0 electron charge
        self.rho_bg = -deposit_charge(p, self.part["x"], self.part["y"]) if p.naive else None

    def deposit(self):
        pt = self.part
        x0, y0 = pt["x"], pt["y"]
        pt["x"], pt["y"] = position_update(self.p, pt["x"], pt["y"], pt["v"])
        vj = 2.0 * pt["v"] - pt["vprev"] if self.p.jvstar else pt["v"]
        if self.p.dirk_substep:
            _, _, cc = self.p.tableau()
            self.J = np.stack([deposit_current(self.p, *stage_positions(self.p, x0, y0, pt["v"], ci), vj)
                               for ci in cc])
        else:
            self.J = deposit_current(self.p, pt["x"], pt["y"], vj)
        if self.p.naive:
            self.rho = deposit_charge(self.p, pt["x"], pt["y"]) + self.rho_bg
        return self.J

    def solve(self):
        if self.p.dirk_substep:
            Jh = np.stack([[spectral.fft2(Ji[c]) for c in range(3)] for Ji in self.J])
        else:
            Jh = np.stack([spectral.fft2(self.J[c]) for c in range(3)])
        rho_h = spectral.fft2(self.rho) if self.p.naive else None
        self.hist, phi_t, A_new = field_update(self.p, self.hist, Jh, rho_h)
        self.fields = gradient_fields(self.p, phi_t, A_new)
        return self.fields

    def gather_push(self):
        pt = self.part
        g = gather(self.p, self.fields, pt["x"], pt["y"])
        Pn, vn = push(self.p, pt["P"], pt["v"], pt["vprev"], g)
        pt["P"], pt["vprev"], pt["v"] = Pn, pt["v"], vn
        self.n += 1

    def step(self, nsteps=1):
        for _ in range(nsteps):
            self.deposit()
            self.solve()
            self.gather_push()
