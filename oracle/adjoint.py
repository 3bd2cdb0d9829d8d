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
round-off, and the gradients equal central finite differences of the same
forward.
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


def run(pr, x, y, P, nsteps):
    """Forward from x^0, P^0 (A^0 = 0, v^{-1} = v^0, cold history)."""
    p = pr.p
    v = velocity(pr, P, torch.zeros_like(P))
    vp = v
    hist = cold_history(pr)
    for _ in range(nsteps):
        x = wrap(x + v[:, 0] * p.dt, p.lx)
        y = wrap(y + v[:, 1] * p.dt, p.ly)
        J = deposit(pr, x, y, v)
        Jh = torch.stack([torch.fft.rfft2(J[c]) for c in range(3)])
        hist, phi, A = bdf_update(pr, hist, Jh)
        F = fields(pr, phi, A)
        g = gather(pr, F, x, y)
        P, vn = push(pr, P, v, vp, g)
        vp, v = v, vn
    return dict(x=x, y=y, P=P, v=v, vprev=vp, hist=hist)


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
    return float(W), gx.numpy(), gy.numpy(), gP.numpy()


def loss(p: pic.Params, x, y, P, nsteps):
    pr = Problem(p)
    with torch.no_grad():
        out = run(pr, torch.tensor(x, dtype=T), torch.tensor(y, dtype=T), torch.tensor(P, dtype=T), nsteps)
        return float(energy(pr, out["hist"]))
