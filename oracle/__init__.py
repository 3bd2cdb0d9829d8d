"""Plain FP64 CPU oracle for the gauge-conserving PIC step (arXiv 2410.18414).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library and does not import it.

Every function is written from the paper's equations, in the paper's order and
notation, in float64, with no blocking, fusion or reordering beyond what the
equations state.  Library primitives used as single steps: ``numpy.fft`` (the
FFT the paper inverts the modified Helmholtz operator with, Sec. 3.1 and
Sec. 4.1) and ``numpy.bincount`` (an ordered sum).

Modules
  bspline     -- centred cardinal B-spline shape function (Sec. 2.2, Sec. 4.1)
  spectral    -- wavenumbers, spectral derivative and Laplacian symbols (Sec. 4.1)
  schemes     -- BDF-k coefficients and C = a*a (Sec. 3.2, Lemma 3.5, Table 1),
                 DIRK-2 tableau (Sec. 5)
  pic         -- Algorithm 1: deposit, continuity, field update (BDF-k, implicit
                 CDF-2, DIRK-2), spectral gradients, gather, IAEM push
  diagnostics -- gauge residual, Gauss residual, charge, field energy

Readings of passages the paper leaves silent or prints garbled are listed in
each function's docstring.
"""

from . import bspline, spectral, schemes, pic, diagnostics  # noqa: F401
