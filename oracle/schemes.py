"""Time-stepper coefficients (oracle; test infrastructure only).

BDF-k (Sec. 3.2): the first derivative is (1/dt) * sum_j a_j u^{n-j}, and the
time-consistent second derivative is that operator applied twice, whose
coefficients are C = a * a (discrete self-convolution; Lemma on the BDF-k
coefficient structure and Table 1).

The a_j are generated from the backward-difference series
    dt * d/dt  =  sum_{j=1}^{k} (1/j) nabla^j ,  nabla u^n = u^n - u^{n-1},
which is the textbook definition of BDF-k.  The paper prints BDF-2 normalised
by a_0 (first derivative 1, -4/3, 1/3 over (2/3) dt; second 1, -8/3, 22/9,
-8/9, 1/9 over ((2/3) dt)^2, remark closing Sec. 3.2); that is the same
operator divided through by a_0 = 3/2.

DIRK-2 (Sec. 5, the Qin-Zhang tableau).  Reading: the printed tableau is
garbled (its abscissae 1/4, 1/4 do not equal its row sums 1/2, 3/4).  The
two-stage Qin-Zhang symplectic DIRK is used:
    c = (1/4, 3/4),  A = [[1/4, 0], [1/2, 1/4]],  b = (1/2, 1/2),
whose stability function ((1 + z/4)/(1 - z/4))^2 has modulus one on the
imaginary axis, matching the paper's remarks that DIRK-2 is dispersive with
no diffusion.
"""

from fractions import Fraction
from math import comb

import numpy as np


def bdf_a_exact(k):
    """BDF-k coefficients a_0..a_k as exact fractions (step dt)."""
    if not 1 <= k <= 6:
        raise ValueError("BDF order must be 1..6")
    a = [Fraction(0)] * (k + 1)
    for j in range(1, k + 1):
        for i in range(j + 1):
            a[i] += Fraction(1, j) * (-1) ** i * comb(j, i)
    return a


def bdf_a(k):
    return np.array([float(v) for v in bdf_a_exact(k)])


def bdf_C(k):
    """C_0..C_{2k} of the second derivative: C = a * a (Table 1)."""
    a = bdf_a(k)
    return np.convolve(a, a)


def bdf_C_exact(k):
    a = bdf_a_exact(k)
    C = [Fraction(0)] * (2 * k + 1)
    for i in range(k + 1):
        for j in range(k + 1):
            C[i + j] += a[i] * a[j]
    return C


# Qin-Zhang two-stage DIRK (reading stated in the module docstring)
DIRK2_A = np.array([[0.25, 0.0], [0.5, 0.25]])
DIRK2_B = np.array([0.5, 0.5])
DIRK2_C = np.array([0.25, 0.75])


def dirk_composed(b):
    """The s-stage DIRK that composes s implicit-midpoint substeps of lengths
    b_i h in sequence: a_ij = b_j for j < i, a_ii = b_i / 2, c_i = sum_j a_ij.
    Symplectic for any weights; b = (1/2, 1/2) is the Qin-Zhang tableau above."""
    b = np.asarray(b, np.float64)
    s = len(b)
    A = np.zeros((s, s))
    for i in range(s):
        A[i, :i] = b[:i]
        A[i, i] = 0.5 * b[i]
    return A, b, A.sum(1)


# DIRK-3 (general s-stage DIRK of Sec. 3.3 with s = 3): the composition with
# the symmetric fourth-order "triple jump" weights b_1 = b_3 = 1/(2 - 2^{1/3}),
# b_2 = 1 - 2 b_1 (Yoshida's construction); stability function
# prod_i (1 + b_i z/2)/(1 - b_i z/2), modulus one on the imaginary axis.
_W1 = 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))
DIRK3_A, DIRK3_B, DIRK3_C = dirk_composed([_W1, 1.0 - 2.0 * _W1, _W1])


def dirk_tableau(scheme):
    return (DIRK2_A, DIRK2_B, DIRK2_C) if scheme == "dirk2" else (DIRK3_A, DIRK3_B, DIRK3_C)
