"""Normalized spectral max-norm error (oracle; test infrastructure).

Sec. 6, eq. error_norm_r_norm:
  E_{R_norm} = max_{m<=R_norm, m<=n<=R_norm} |phi_n^m - ref_n^m|
               / max_{m<=R_norm, m<=n<=R_norm} |ref_n^m|.
For the geopotential the mean mode (0,0) carries sqrt(2) Phibar and would hide
every other error in the denominator, so ``exclude_mean=True`` drops the (0,0)
slot from both maxima (the literal norm is ``exclude_mean=False``).
"""

import numpy as np

from . import sht


def error_norm(phi, ref, T, R_norm=None, exclude_mean=False):
    R = T if R_norm is None else min(R_norm, T)
    m, n = sht.mn_arrays(T)
    keep = (m <= R) & (n <= R)
    if exclude_mean:
        keep &= ~((m == 0) & (n == 0))
    num = np.abs(phi[..., keep] - ref[..., keep]).max()
    den = np.abs(ref[..., keep]).max()
    return num / den if den > 0 else num
