"""Gaussian grid of the spectral transform method (oracle; test infrastructure).

Sec. 3 (spectral transform method): the physical grid uses Gaussian latitudes
mu = sin(phi), i.e. the roots of the Legendre polynomial P_nlat, with the
Gauss-Legendre weights, and uniformly spaced longitudes lambda_k = 2 pi k/nlon.
Latitudes are ordered north to south (mu descending).
"""

import numpy as np


def legendre_poly_and_derivative(n, x):
    """P_n(x) and P_n'(x) (unnormalized Legendre polynomial) by the
    three-term recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}."""
    x = np.asarray(x, dtype=np.float64)
    p0 = np.ones_like(x)
    if n == 0:
        return p0, np.zeros_like(x)
    p1 = x.copy()
    for k in range(1, n):
        p0, p1 = p1, ((2 * k + 1) * x * p1 - k * p0) / (k + 1)
    # derivative from (1 - x^2) P_n' = n (P_{n-1} - x P_n)
    dp = n * (p0 - x * p1) / (1.0 - x * x)
    return p1, dp


def gauss_latitudes(nlat):
    """Gauss-Legendre nodes mu_j (descending, north to south) and weights w_j.

    Newton iteration on P_nlat from the classical cosine initial guess;
    weights w_j = 2 / ((1 - mu_j^2) P_nlat'(mu_j)^2).  Sum of weights is 2.
    """
    i = np.arange(nlat, dtype=np.float64)
    x = np.cos(np.pi * (i + 0.75) / (nlat + 0.5))
    for _ in range(100):
        p, dp = legendre_poly_and_derivative(nlat, x)
        dx = p / dp
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    p, dp = legendre_poly_and_derivative(nlat, x)
    w = 2.0 / ((1.0 - x * x) * dp * dp)
    order = np.argsort(-x)
    return x[order], w[order]


def longitudes(nlon):
    """lambda_k = 2 pi k / nlon, k = 0..nlon-1."""
    return 2.0 * np.pi * np.arange(nlon, dtype=np.float64) / nlon
