"""Scalar spherical-harmonic transform (oracle; test infrastructure).

Sec. 3, eq. (spectral_to_physical_space): xi(lambda, mu) is the sum over
zonal wavenumbers r and total wavenumbers s >= |r| of xi_s^r P_s^r(mu) e^{i r lambda},
triangular truncation S(r) = R.  Only r >= 0 is stored (the field is real, so
xi_s^{-r} = conj(xi_s^r) and Im xi_s^0 = 0).  Truncation T is the largest
wavenumber kept: m = 0..T, n = m..T, stored m-major in K = (T+1)(T+2)/2 slots.

The transform has the two steps of Sec. 3: a Fourier transform in longitude
(numpy.fft, a library primitive) and a Gauss-Legendre quadrature in latitude.
"""

import numpy as np

from . import grid as _grid
from . import legendre as _leg


def ncoef(T):
    return (T + 1) * (T + 2) // 2


def offset(T, m):
    """Index of (m, n=m) in the m-major layout."""
    return m * (T + 1) - m * (m - 1) // 2


def mn_arrays(T):
    """m and n of every slot of the m-major layout."""
    ms, ns = [], []
    for m in range(T + 1):
        for n in range(m, T + 1):
            ms.append(m)
            ns.append(n)
    return np.array(ms), np.array(ns)


def index(T, m, n):
    return offset(T, m) + (n - m)


class Grid:
    """Gaussian grid and Legendre tables for truncation T on nlat x nlon."""

    def __init__(self, T, nlat, nlon):
        if nlat < T + 1 or nlon < 2 * T + 1:
            raise ValueError("grid too coarse for truncation")
        self.T, self.nlat, self.nlon = T, nlat, nlon
        self.mu, self.w = _grid.gauss_latitudes(nlat)
        self.lam = _grid.longitudes(nlon)
        self.P = _leg.p_tables(T, self.mu)      # rows n = m..T+1
        self.H = _leg.h_tables(T, self.mu, self.P)  # rows n = m..T
        self.K = ncoef(T)
        self.m_of, self.n_of = mn_arrays(T)


def legendre_synthesis(g, spec):
    """Fourier coefficients X[j, m] = sum_n xi_n^m P_n^m(mu_j), m = 0..T."""
    T = g.T
    X = np.zeros((g.nlat, T + 1), dtype=np.complex128)
    for m in range(T + 1):
        o = offset(T, m)
        X[:, m] = spec[o:o + T + 1 - m] @ g.P[m][: T + 1 - m]
    return X


def fourier_synthesis(g, X):
    """xi(lambda_k, mu_j) = X_0 + 2 Re sum_{m>=1} X_m e^{i m lambda_k}."""
    c = np.zeros((g.nlat, g.nlon // 2 + 1), dtype=np.complex128)
    c[:, : g.T + 1] = X * g.nlon
    c[:, 0] = c[:, 0].real
    return np.fft.irfft(c, n=g.nlon, axis=1)


def fourier_analysis(g, field):
    """X[j, m] = (1/nlon) sum_k xi(lambda_k, mu_j) e^{-i m lambda_k}, m = 0..T."""
    c = np.fft.rfft(field, axis=1) / g.nlon
    return c[:, : g.T + 1]


def legendre_analysis(g, X):
    """xi_n^m = sum_j w_j P_n^m(mu_j) X_m(mu_j); Im xi_n^0 set to 0."""
    T = g.T
    spec = np.zeros(g.K, dtype=np.complex128)
    for m in range(T + 1):
        o = offset(T, m)
        spec[o:o + T + 1 - m] = g.P[m][: T + 1 - m] @ (g.w * X[:, m])
    spec[: T + 1] = spec[: T + 1].real
    return spec


def synthesis(g, spec):
    """Spectral coefficients [K] -> grid [nlat, nlon] (lat north to south)."""
    return fourier_synthesis(g, legendre_synthesis(g, spec))


def analysis(g, field):
    """Grid [nlat, nlon] -> spectral coefficients [K]."""
    return legendre_analysis(g, fourier_analysis(g, field))
