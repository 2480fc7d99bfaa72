"""Space-time transfer operators and the FAS correction (oracle; test infrastructure).

Sec. 5.3 (construction of the coarse level):
  restriction     R = (R^s)(R^t): in time Pi^c_f with (Pi^c_f)_ij = l_j^f(t_i^c)
                  (eq. time_restriction), then in space the truncation matrix
                  D^c_f that keeps the coefficients with m, n <= T_c
                  (eq. space_restriction);
  interpolation   P = (P^t)(P^s): zero-padding P^s = (R^s)^T, then
                  Pi^f_c with (Pi^f_c)_ij = l_j^c(t_i^f) (eq. time_interpolation).
Sec. 5.1.2 (FAS), eq. tau_term_level_l+1 with tau_f = 0:
  tau_c = A_c(R Theta_f) - R A_f(Theta_f)
        = dt [ R (Q_f (x) I) F_f  -  (Q_c (x) I) F_c(R Theta_f) ]
(the Theta terms cancel because R is linear), one K_c-vector per coarse node.

Space-time arrays are [nodes, 3, K] complex128 in the m-major layout.
"""

import numpy as np

from . import sdc, sht


def truncate(x, Tf, Tc):
    """Keep m, n <= Tc of the last axis (m-major, Tf -> Tc)."""
    parts = []
    for m in range(Tc + 1):
        o = sht.offset(Tf, m)
        parts.append(x[..., o:o + Tc + 1 - m])
    return np.concatenate(parts, axis=-1)


def zero_pad(x, Tc, Tf):
    """Inverse of truncate on the kept modes; zeros elsewhere (P^s = (R^s)^T)."""
    out = np.zeros(x.shape[:-1] + (sht.ncoef(Tf),), dtype=x.dtype)
    for m in range(Tc + 1):
        of = sht.offset(Tf, m)
        oc = sht.offset(Tc, m)
        out[..., of:of + Tc + 1 - m] = x[..., oc:oc + Tc + 1 - m]
    return out


def time_restriction(sd_f, sd_c):
    return sdc.lagrange_matrix(sd_f.nodes, sd_c.nodes)


def time_interpolation(sd_c, sd_f):
    return sdc.lagrange_matrix(sd_c.nodes, sd_f.nodes)


def restrict(sd_f, sd_c, Tf, Tc, x_f):
    """R x_f: [Mf+1, ..., Kf] -> [Mc+1, ..., Kc]."""
    Pi = time_restriction(sd_f, sd_c)
    xt = np.einsum("ij,j...->i...", Pi, x_f)
    return truncate(xt, Tf, Tc)


def interpolate(sd_c, sd_f, Tc, Tf, x_c):
    """P x_c: [Mc+1, ..., Kc] -> [Mf+1, ..., Kf]."""
    xs = zero_pad(x_c, Tc, Tf)
    Pi = time_interpolation(sd_c, sd_f)
    return np.einsum("ij,j...->i...", Pi, xs)


def fas_tau(sd_f, sd_c, Tf, Tc, dt, fe_f, fi_f, fe_c, fi_c):
    """tau_c = dt [ R (Q_f F_f) - Q_c F_c ], with F_c evaluated at R Theta_f."""
    int_f = sdc.integral(sd_f, dt, fe_f, fi_f)
    int_c = sdc.integral(sd_c, dt, fe_c, fi_c)
    return restrict(sd_f, sd_c, Tf, Tc, int_f) - int_c
