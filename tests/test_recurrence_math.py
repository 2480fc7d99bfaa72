"""CPU pins of the two-degree Legendre recurrence that the recurrence-mode
kernels evaluate (Sec. 3; PFSH_LEGENDRE_RECURRENCE in include/pfsh.h):

  P_{n+2} = a ((mu^2 - b) P_n - c P_{n-2}),
  a = 1 / (e_{n+1} e_{n+2}), b = e_{n+1}^2 + e_n^2, c = e_n e_{n-1},
  e_n = sqrt((n^2 - m^2) / (4 n^2 - 1)),

restarted every 32 degrees of one parity from the pair (P_{n0-2}, P_{n0}).
The reference is the oracle's 80-bit P_n^m table, itself pinned by
orthonormality under Gauss quadrature (test_oracle_transform.py); the walk is
done in float64 as the kernels do it."""

import numpy as np
import pytest

from oracle import grid, legendre

CHUNK = 32


def _coef(n, m):
    e = lambda k: legendre.eps(k, m) if k > m else 0.0
    return 1.0 / (e(n + 1) * e(n + 2)), e(n + 1) ** 2 + e(n) ** 2, e(n) * e(n - 1)


@pytest.mark.parametrize("T,nlat", [(40, 42), (255, 384)])
def test_two_degree_recurrence_chunks_reproduce_the_table(T, nlat):
    mu, _ = grid.gauss_latitudes(nlat)
    mu = mu[: nlat // 2]
    P = legendre.p_tables(T, mu)
    worst = 0.0
    for m in (0, 1, T // 3, T // 2 + 1, T - 2):
        for p in (0, 1):
            n_deg = (T + 1 - m - p) // 2 + 1           # degrees m+p, m+p+2, ... <= T+1
            for c0 in range(0, n_deg, CHUNK):
                d0 = p + 2 * c0                        # n0 - m
                s0 = P[m][d0 - 2] if d0 >= 2 else np.zeros_like(mu)
                s1 = P[m][d0].copy()
                for t in range(1, min(CHUNK, n_deg - c0)):
                    n = m + d0 + 2 * (t - 1)
                    a, b, c = _coef(n, m)
                    s0, s1 = s1, a * ((mu * mu - b) * s1 - c * s0)
                    ref = P[m][d0 + 2 * t]
                    scale = np.abs(P[m]).max(axis=0) + 1e-300
                    worst = max(worst, float((np.abs(s1 - ref) / scale).max()))
    # float64 walk of at most 31 steps: each step rounds a few times and the
    # three-term recurrence carries those errors forward without damping, so
    # the error grows about linearly along the chunk.  Measured at T255: 1.0e-13
    # of the column scale (the one-degree recurrence over the same 62
    # degrees: 6.5e-14), 4.5e-14 with 16-degree chunks.
    assert worst <= 2e-13, worst


def test_planted_sign_error_in_the_recurrence_is_caught():
    """A flipped sign of the c term (the plausible slip) leaves the first step
    of a chunk from P_{n0-2} = 0 intact but breaks every later one."""
    T, nlat = 40, 42
    mu, _ = grid.gauss_latitudes(nlat)
    mu = mu[: nlat // 2]
    P = legendre.p_tables(T, mu)
    m, p = 3, 0
    s0, s1 = np.zeros_like(mu), P[m][0].copy()
    for t in range(1, 6):
        a, b, c = _coef(m + 2 * (t - 1), m)
        s0, s1 = s1, a * ((mu * mu - b) * s1 + c * s0)
    assert np.abs(s1 - P[m][10]).max() > 1e-3 * np.abs(P[m][10]).max()


def test_restart_pair_below_the_order_is_zero():
    """For n0 = m (+p) the pair's first value P_{n0-2} lies below the order: the
    coefficient c vanishes there, so the value 0 stored for it is exact."""
    for m in (0, 5, 30):
        for p in (0, 1):
            _, _, c = _coef(m + p, m)
            assert c == 0.0
