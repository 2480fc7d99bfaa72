"""FP64 CPU oracle for the PFASST-SH hot path (test infrastructure only).

This package is the plain, slow, obviously-correct reference for what the GPU
library computes.  It is test infrastructure: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The product path (``paper_1904_05988_amd``) never imports it and
shares no code, tables or constants with it.

Everything here is NumPy in float64 (Legendre seeds are run in the x87
80-bit ``longdouble`` so that P_m^m does not underflow at high order), follows
the paper's definitions step by step, and is pinned against closed forms,
invariants and library routines in ``tests/test_oracle_*.py``.

Modules
  grid      Gaussian latitudes and weights, longitudes            (Sec. 3)
  legendre  normalized associated Legendre P_n^m and H_n^m tables  (Sec. 3)
  sht       scalar spherical-harmonic synthesis / analysis         (Sec. 3)
  swe       shallow-water operators L, N, implicit solve           (Sec. 2, 5.4)
  sdc       Lobatto nodes, Q / Q_E / Q_I, IMEX SDC sweep, residual  (Sec. 5.1.1)
  transfer  space-time restriction / interpolation, FAS tau        (Sec. 5.1.2, 5.3)
  pfasst    predictor and PFASST iteration with explicit mailboxes (Sec. 5.2)
  metrics   normalized spectral max-norm error                     (Sec. 6)
"""

from . import grid, legendre, sht, swe, sdc, transfer, pfasst, metrics  # noqa: F401
