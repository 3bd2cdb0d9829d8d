"""Spectral symbols on the periodic grid (oracle; test infrastructure only).

All spatial derivatives are spectral and consistent with the FFT inverse of
the modified Helmholtz operator (Sec. 4.1, the paragraph after the IAEM
equations; the operator L = I - Laplacian/alpha^2 is defined in Sec. 3.1).

Layout: real fields are arrays [ny, nx] (x is the last, fastest axis); their
transforms are numpy.fft.rfft2 arrays [ny, nx//2 + 1].

Reading (the paper is silent on the Nyquist mode): the first-derivative symbol
i*k is set to zero at the Nyquist index of each axis, and the Laplacian symbol
is built from the same k, -(kx_d^2 + ky_d^2), so that div(grad) equals the
Laplacian exactly, which the Gauss-law theorems use.
"""

import numpy as np


def wavenumbers(nx, ny, lx, ly):
    """Return (kx_d, ky_d) broadcastable to [ny, nx//2+1], Nyquist zeroed."""
    kx = 2.0 * np.pi * np.fft.rfftfreq(nx, d=lx / nx)
    ky = 2.0 * np.pi * np.fft.fftfreq(ny, d=ly / ny)
    if nx % 2 == 0:
        kx[nx // 2] = 0.0
    if ny % 2 == 0:
        ky[ny // 2] = 0.0
    return kx[None, :], ky[:, None]


def symbols(nx, ny, lx, ly):
    """Return (ikx, iky, lap) symbols on the half spectrum."""
    kx, ky = wavenumbers(nx, ny, lx, ly)
    ikx = 1j * kx * np.ones((ny, 1))
    iky = 1j * ky * np.ones((1, nx // 2 + 1))
    lap = -(kx ** 2 + ky ** 2)
    return ikx, iky, lap


def fft2(f):
    return np.fft.rfft2(f)


def ifft2(fh, nx, ny):
    return np.fft.irfft2(fh, s=(ny, nx))
