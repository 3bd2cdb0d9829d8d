"""Reference gradients of the PIC step by automatic differentiation
(oracle; test infrastructure only).

The forward step is Algorithm 1 again (see oracle/pic.py for the readings),
written with plain PyTorch CPU float64 operations so that torch.autograd gives
the exact derivative of the discrete map: deposit by index_add, numpy-free FFTs
(torch.fft), the BDF-k update of Sec. 3.2, spectral gradients, gather, IAEM
push (Sec. 4.1).  Only BDF-k is provided (the stepper of the adjoint workload).

Loss: the field energy of the newest level (Sec. 2.2, E = -grad phi - dA/dt,
B = curl A) with the BDF-k time derivative of Sec. 3.2:
    W = (dx dy / 2) sum_mesh (eps0 |E|^2 + |B|^2 / mu0),
    E = -grad phi^n - (1/dt) sum_j a_j A^{n-j},  B = curl A^n.

Pins (tests/test_oracle_adjoint.py): the forward equals the numpy oracle to
round-off; the gradients equal central finite differences of the same
forward; the one-step vector-Jacobian product passes the dot-product test
against directional differences of the numpy oracle's step.
"""

import numpy as np
import torch

from . import pic, schemes

T = torch.float64


def _M(m, t):
    """Centred cardinal B-spline of degree m as torch piecewise polynomial in |t|."""
    a = t.abs()
    z = torch.zeros_like(a)
    if m == 1:
        return torch.where(a < 1, 1 - a, z)
    if m == 2:
        return torch.where(a < 0.5, 0.75 - a * a, torch.where(a < 1.5, 0.5 * (1.5 - a) ** 2, z))
    if m == 3:
        return torch.where(a < 1, 2.0 / 3.0 - a * a + 0.5 * a ** 3,
                           torch.where(a < 2, (2 - a) ** 3 / 6.0, z))
    raise ValueError(m)


def _stencil(m, xi):
    base = torch.floor(xi.detach()).to(torch.int64)
    offs = torch.arange(-1, 3, dtype=torch.int64)
    g = base[:, None] + offs[None, :]
    return g, _M(m, g.to(T) - xi[:, None])


class Problem:
    """Grid, constants and spectral symbols (torch tensors) of one run."""

    def __init__(self, p: pic.Params):
        self.p = p
        self.ikx = torch.tensor(p.ikx * np.ones(p.spec_shape), dtype=torch.complex128)
        self.iky = torch.tensor(p.iky * np.ones(p.spec_shape), dtype=torch.complex128)
        self.lap = torch.tensor(p.lap * np.ones(p.spec_shape), dtype=T)
        self.a = schemes.bdf_a(p.bdf_order)
        self.C = schemes.bdf_C(p.bdf_order)


def velocity(pr, P, A):
    p = pr.p
    u = P - p.q * A
    s = torch.sqrt(p.c ** 2 * (u * u).sum(1) + (p.m * p.c ** 2) ** 2)
    return p.c ** 2 * u / s[:, None]


def wrap(x, L):
    x = x - L * torch.floor(x.detach() / L)
    return torch.where(x.detach() >= L, x - L, x)


def deposit(pr, x, y, v):
    p = pr.p
    gx, wx = _stencil(p.degree, x / p.dx)
    gy, wy = _stencil(p.degree, y / p.dy)
    n = p.nx * p.ny
    J = torch.zeros(3, n, dtype=T)
    qv = p.q * v
    for a in range(4):
        for b in range(4):
            idx = (gy[:, b] % p.ny) * p.nx + (gx[:, a] % p.nx)
            w = wx[:, a] * wy[:, b] / (p.dx * p.dy)
            for c in range(3):
                J[c] = J[c].index_add(0, idx, w * qv[:, c])
    return J.reshape(3, p.ny, p.nx)


def gather(pr, F, x, y):
    p = pr.p
    gx, wx = _stencil(p.degree, x / p.dx)
    gy, wy = _stencil(p.degree, y / p.dy)
    Ff = F.reshape(F.shape[0], -1)
    out = torch.zeros(x.shape[0], F.shape[0], dtype=T)
    for a in range(4):
        for b in range(4):
            idx = (gy[:, b] % p.ny) * p.nx + (gx[:, a] % p.nx)
            out = out + (wx[:, a] * wy[:, b])[:, None] * Ff[:, idx].T
    return out


def bdf_update(pr, hist, Jh):
    p = pr.p
    a, C = pr.a, pr.C
    k = p.bdf_order
    div = pr.ikx * Jh[0] + pr.iky * Jh[1]
    rho = -(sum(a[j] * hist["rho"][j - 1] for j in range(1, k + 1)) + p.dt * div) / a[0]
    alpha2 = (a[0] / (p.c * p.dt)) ** 2
    Lh = 1.0 - pr.lap / alpha2
    phi = (rho / (p.eps0 * alpha2) - sum(C[i] / C[0] * hist["phi"][i - 1]
                                           for i in range(1, 2 * k + 1))) / Lh
    A = (p.mu0 * Jh / alpha2 - sum(C[i] / C[0] * hist["A"][i - 1] for i in range(1, 2 * k + 1))) / Lh
    new = dict(rho=[rho] + hist["rho"][:-1], phi=[phi] + hist["phi"][:-1], A=[A] + hist["A"][:-1])
    return new, phi, A


def fields(pr, phi, A):
    p = pr.p
    spec = [pr.ikx * phi, pr.iky * phi, A[0], A[1], A[2], pr.ikx * A[0], pr.ikx * A[1],
            pr.ikx * A[2], pr.iky * A[0], pr.iky * A[1], pr.iky * A[2]]
    return torch.stack([torch.fft.irfft2(f, s=(p.ny, p.nx)) for f in spec])


def push(pr, P, v, vp, g):
    p = pr.p
    vs = 2 * v - vp
    Fx = -g[:, 0] + vs[:, 0] * g[:, 5] + vs[:, 1] * g[:, 6] + vs[:, 2] * g[:, 7]
    Fy = -g[:, 1] + vs[:, 0] * g[:, 8] + vs[:, 1] * g[:, 9] + vs[:, 2] * g[:, 10]
    Pn = torch.stack([P[:, 0] + p.q * Fx * p.dt, P[:, 1] + p.q * Fy * p.dt, P[:, 2]], 1)
    return Pn, velocity(pr, Pn, g[:, 2:5])


def cold_history(pr):
    p = pr.p
    z = lambda: torch.zeros(p.spec_shape, dtype=torch.complex128)  # noqa: E731
    k = p.bdf_order
    return dict(rho=[z() for _ in range(k)], phi=[z() for _ in range(2 * k)],
                A=[torch.zeros((3,) + p.spec_shape, dtype=torch.complex128) for _ in range(2 * k)])


def step_from(pr, x, y, P, v, vp, hist):
    """One step of Algorithm 1 from the state (x^n, P^n, v^n, v^{n-1}, history)."""
    p = pr.p
    x = wrap(x + v[:, 0] * p.dt, p.lx)
    y = wrap(y + v[:, 1] * p.dt, p.ly)
    J = deposit(pr, x, y, v)
    Jh = torch.stack([torch.fft.rfft2(J[c]) for c in range(3)])
    hist, phi, A = bdf_update(pr, hist, Jh)
    F = fields(pr, phi, A)
    g = gather(pr, F, x, y)
    P, vn = push(pr, P, v, vp, g)
    return x, y, P, vn, v, hist


def run(pr, x, y, P, nsteps):
    """Forward from x^0, P^0 (A^0 = 0, v^{-1} = v^0, cold history)."""
    v = velocity(pr, P, torch.zeros_like(P))
    vp = v
    hist = cold_history(pr)
    for _ in range(nsteps):
        x, y, P, v, vp, hist = step_from(pr, x, y, P, v, vp, hist)
    return dict(x=x, y=y, P=P, v=v, vprev=vp, hist=hist)


def _hist_leaves(hist):
    """numpy history dict -> torch leaves (requires_grad) in the same structure."""
    mk = lambda a: torch.tensor(a, dtype=torch.complex128, requires_grad=True)  # noqa: E731
    return dict(rho=[mk(a) for a in hist["rho"]], phi=[mk(a) for a in hist["phi"]],
                A=[mk(a) for a in hist["A"]])


def _hist_flat(hist):
    """History dict -> list of per-field tensors in the exported order (rho levels,
    phi levels, then A levels with their three components)."""
    out = list(hist["rho"]) + list(hist["phi"])
    for A in hist["A"]:
        out += [A[0], A[1], A[2]]
    return out


def _pairing(lam, z):
    """Real inner product <lam, z> = sum Re(conj(lam) z)."""
    if torch.is_complex(z):
        return (torch.conj(lam) * z).real.sum()
    return (lam * z).sum()


def step_vjp(p: pic.Params, part, hist, lam_part, lam_hist):
    """(dS^{n+1}/dS^n)^T lambda for one step from the numpy state (part: x, y,
    P, v, vprev as in oracle/pic.py; hist: its history dict).  lam_part has
    the same keys; lam_hist is [nfield, ny, nx/2+1] complex in the exported
    order.  Complex adjoints use dL/dRe + i dL/dIm (torch's convention).
    Returns (lam_part_n, lam_hist_n) in the same forms."""
    pr = Problem(p)
    t = lambda a: torch.tensor(np.asarray(a), dtype=T, requires_grad=True)  # noqa: E731
    x, y, P, v, vp = t(part["x"]), t(part["y"]), t(part["P"]), t(part["v"]), t(part["vprev"])
    h = _hist_leaves(hist)
    xo, yo, Po, vo, vpo, ho = step_from(pr, x, y, P, v, vp, h)
    L = 0.0
    for key, z in (("x", xo), ("y", yo), ("P", Po), ("v", vo), ("vprev", vpo)):
        L = L + _pairing(torch.tensor(np.asarray(lam_part[key]), dtype=T), z)
    lh = torch.tensor(np.asarray(lam_hist), dtype=torch.complex128)
    for f, z in enumerate(_hist_flat(ho)):
        L = L + _pairing(lh[f], z)
    # A levels are leaves of shape (3, ny, nxh): differentiate the leaves, then split
    leaves = [x, y, P, v, vp] + list(h["rho"]) + list(h["phi"]) + list(h["A"])
    g = torch.autograd.grad(L, leaves, allow_unused=True)
    g = [torch.zeros_like(a) if gi is None else gi for a, gi in zip(leaves, g)]
    out = dict(x=g[0].numpy(), y=g[1].numpy(), P=g[2].numpy(), v=g[3].numpy(), vprev=g[4].numpy())
    k = p.bdf_order
    rho_g, phi_g, A_g = g[5:5 + k], g[5 + k:5 + 3 * k], g[5 + 3 * k:]
    flat = [a.numpy() for a in rho_g] + [a.numpy() for a in phi_g]
    for A in A_g:
        flat += [A[0].numpy(), A[1].numpy(), A[2].numpy()]
    return out, np.stack(flat)


def energy_hist_grad(p: pic.Params, hist):
    """dW/d(history) of the field energy of the newest level, [nfield, ny, nx/2+1]."""
    pr = Problem(p)
    h = _hist_leaves(hist)
    W = energy(pr, h)
    leaves = list(h["rho"]) + list(h["phi"]) + list(h["A"])
    g = torch.autograd.grad(W, leaves, allow_unused=True)
    g = [torch.zeros_like(a) if gi is None else gi for a, gi in zip(leaves, g)]
    k = p.bdf_order
    flat = [a.numpy() for a in g[:3 * k]]
    for A in g[3 * k:]:
        flat += [A[0].numpy(), A[1].numpy(), A[2].numpy()]
    return np.stack(flat)


def energy(pr, hist):
    """W of the newest level (BDF-k time derivative of A)."""
    p = pr.p
    a = pr.a
    phi = hist["phi"][0]
    A0 = hist["A"][0]
    dA = sum(a[j] * hist["A"][j] for j in range(p.bdf_order + 1)) / p.dt
    Eh = [-pr.ikx * phi - dA[0], -pr.iky * phi - dA[1], -dA[2]]
    Bh = [pr.iky * A0[2], -pr.ikx * A0[2], pr.ikx * A0[1] - pr.iky * A0[0]]
    r = lambda f: torch.fft.irfft2(f, s=(p.ny, p.nx))  # noqa: E731
    E2 = sum(r(e) ** 2 for e in Eh)
    B2 = sum(r(b) ** 2 for b in Bh)
    return 0.5 * p.dx * p.dy * (p.eps0 * E2 + B2 / p.mu0).sum()


def loss_and_grad(p: pic.Params, x, y, P, nsteps):
    """W after nsteps and its gradient with respect to the initial x, y, P."""
    pr = Problem(p)
    xt = torch.tensor(x, dtype=T, requires_grad=True)
    yt = torch.tensor(y, dtype=T, requires_grad=True)
    Pt = torch.tensor(P, dtype=T, requires_grad=True)
    out = run(pr, xt, yt, Pt, nsteps)
    W = energy(pr, out["hist"])
    gx, gy, gP = torch.autograd.grad(W, (xt, yt, Pt))
    return float(W.detach()), gx.detach().numpy(), gy.detach().numpy(), gP.detach().numpy()


def loss(p: pic.Params, x, y, P, nsteps):
    pr = Problem(p)
    with torch.no_grad():
        out = run(pr, torch.tensor(x, dtype=T), torch.tensor(y, dtype=T), torch.tensor(P, dtype=T), nsteps)
        return float(energy(pr, out["hist"]))
