"""Centred cardinal B-spline shape functions (oracle; test infrastructure only).

The paper deposits J and gathers fields with tensor products of symmetric
B-splines (Sec. 2.2, after the PIC current density; Sec. 4.1, the paragraph on
the current weighting), but it does not print the spline.  The reading used
here: the centred cardinal B-spline M_m of degree m is the (m+1)-fold
convolution of the unit box on [-1/2, 1/2); nodes sit at i*dx, and a particle
at x contributes with weight M_m((x_i - x)/dx) * M_m((y_j - y)/dy) / (dx*dy).

M_m is written below as its piecewise polynomial in |t| (the plain definition),
not as per-node weight formulas.
"""

import numpy as np

# support radius (m+1)/2 of M_m
SUPPORT = {0: 0.5, 1: 1.0, 2: 1.5, 3: 2.0, 4: 2.5, 5: 3.0}


def M(m, t):
    """Centred cardinal B-spline of degree m (0..3) evaluated at t (array)."""
    a = np.abs(np.asarray(t, dtype=np.float64))
    if m == 0:
        return np.where(a < 0.5, 1.0, 0.0)
    if m == 1:
        return np.where(a < 1.0, 1.0 - a, 0.0)
    if m == 2:
        b = 1.5 - a
        return np.where(a < 0.5, 0.75 - a * a, np.where(a < 1.5, 0.5 * b * b, 0.0))
    if m == 3:
        b = 2.0 - a
        return np.where(a < 1.0, 2.0 / 3.0 - a * a + 0.5 * a * a * a,
                        np.where(a < 2.0, b * b * b / 6.0, 0.0))
    a2 = a * a
    if m == 4:
        return np.where(a < 0.5, 115.0 / 192.0 - 0.625 * a2 + 0.25 * a2 * a2,
                        np.where(a < 1.5, (55.0 + 20.0 * a - 120.0 * a2 + 80.0 * a2 * a - 16.0 * a2 * a2) / 96.0,
                                 np.where(a < 2.5, (5.0 - 2.0 * a) ** 4 / 384.0, 0.0)))
    if m == 5:
        return np.where(a < 1.0, 0.55 - 0.5 * a2 + 0.25 * a2 * a2 - a2 * a2 * a / 12.0,
                        np.where(a < 2.0, 17.0 / 40.0 + 0.625 * a - 1.75 * a2 + 1.25 * a2 * a
                                 - 0.375 * a2 * a2 + a2 * a2 * a / 24.0,
                                 np.where(a < 3.0, (3.0 - a) ** 5 / 120.0, 0.0)))
    raise ValueError("spline degree must be 0..5")


def stencil(m, xi):
    """Node indices (unwrapped) and weights M_m(g - xi) for positions xi = x/dx.

    Returns (g, w) of shape (N, 4) for m <= 3 -- the nodes floor(xi)-1 ..
    floor(xi)+2 cover the support |t| < 2 -- and (N, 6) for m = 4, 5 -- the
    nodes floor(xi)-2 .. floor(xi)+3 cover |t| < 3; weights outside the
    support evaluate to zero.
    """
    xi = np.asarray(xi, dtype=np.float64)
    base = np.floor(xi).astype(np.int64)
    offs = np.arange(-1, 3) if m <= 3 else np.arange(-2, 4)
    g = base[:, None] + offs[None, :]
    w = M(m, g - xi[:, None])
    return g, w
