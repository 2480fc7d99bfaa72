"""Normalized associated Legendre functions (oracle; test infrastructure).

Sec. 3: the expansion uses the normalized associated Legendre functions
P_s^r.  The paper does not print the normalization; the reading taken here is
int_{-1}^{1} (P_n^m)^2 dmu = 1 with P_m^m > 0 (no Condon-Shortley phase).

Recurrences (textbook, in the order used):
  P_0^0     = 1/sqrt(2)
  P_m^m     = sqrt((2m+1)/(2m)) sqrt(1-mu^2) P_{m-1}^{m-1}
  P_{m+1}^m = sqrt(2m+3) mu P_m^m
  P_n^m     = (mu P_{n-1}^m - eps_{n-1}^m P_{n-2}^m) / eps_n^m,
              eps_n^m = sqrt((n^2 - m^2) / (4 n^2 - 1))
and H_n^m = (1 - mu^2) dP_n^m/dmu = -n eps_{n+1}^m P_{n+1}^m + (n+1) eps_n^m P_{n-1}^m,
which needs P up to degree T+1.

The sectoral seed P_m^m ~ (1-mu^2)^{m/2} leaves the float64 range near the
poles at high m (about 1e-535 at T255), so the recurrence runs in the x87
80-bit longdouble and the table is rounded to float64 at the end (values
below the float64 range become 0, which is their value to float64 accuracy).
"""

import numpy as np


def eps(n, m):
    """eps_n^m = sqrt((n^2 - m^2)/(4 n^2 - 1)) as float64; 0 for n <= m."""
    return float(_eps_ld(n, m))


def _eps_ld(n, m):
    if n <= m:
        return np.longdouble(0)
    return np.sqrt(np.longdouble(n * n - m * m) / np.longdouble(4 * n * n - 1))


def p_tables(T, mu):
    """P[m] of shape (T+2-m, len(mu)), rows n = m..T+1, float64."""
    x = np.asarray(mu, dtype=np.longdouble)
    s = np.sqrt(np.longdouble(1) - x * x)
    out = []
    pmm = np.full_like(x, np.longdouble(1) / np.sqrt(np.longdouble(2)))
    for m in range(T + 1):
        if m > 0:
            pmm = np.sqrt(np.longdouble(2 * m + 1) / np.longdouble(2 * m)) * s * pmm
        rows = [pmm]
        rows.append(np.sqrt(np.longdouble(2 * m + 3)) * x * pmm)
        for n in range(m + 2, T + 2):
            pn = (x * rows[-1] - _eps_ld(n - 1, m) * rows[-2]) / _eps_ld(n, m)
            rows.append(pn)
        out.append(np.array(rows[: T + 2 - m], dtype=np.float64))
    return out


def h_tables(T, mu, P=None):
    """H[m] of shape (T+1-m, len(mu)), rows n = m..T:
    H_n^m = -n eps_{n+1}^m P_{n+1}^m + (n+1) eps_n^m P_{n-1}^m  (P_{m-1}^m = 0)."""
    if P is None:
        P = p_tables(T, mu)
    out = []
    for m in range(T + 1):
        Pm = P[m]
        rows = []
        for n in range(m, T + 1):
            h = -n * float(_eps_ld(n + 1, m)) * Pm[n + 1 - m]
            if n - 1 >= m:
                h = h + (n + 1) * float(_eps_ld(n, m)) * Pm[n - 1 - m]
            rows.append(h)
        out.append(np.array(rows))
    return out
