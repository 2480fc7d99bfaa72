"""Pins of the oracle's grid, Legendre tables and scalar transform.

Each pin comes from outside the oracle: a library routine (numpy leggauss,
scipy lpmv), a closed form, or brute-force term-by-term evaluation.
"""

import math

import numpy as np
import pytest

from oracle import grid, legendre, sht
from tests._direct import evaluate, pnm

T_SMALL = 15
NLAT, NLON = 24, 48


@pytest.fixture(scope="module")
def g():
    return sht.Grid(T_SMALL, NLAT, NLON)


@pytest.mark.parametrize("nlat", [6, 24, 48, 192])
def test_gauss_nodes_match_numpy(nlat):
    mu, w = grid.gauss_latitudes(nlat)
    x, wx = np.polynomial.legendre.leggauss(nlat)
    assert np.all(np.diff(mu) < 0)
    np.testing.assert_allclose(mu, x[::-1], atol=2e-15)
    # numpy.leggauss weights carry up to ~6e-11 relative error near the poles at
    # nlat=192 (its own accuracy); the exact-moment test below is the tight pin
    np.testing.assert_allclose(w, wx[::-1], rtol=1e-10, atol=1e-16)


@pytest.mark.parametrize("nlat", [24, 96])
def test_gauss_quadrature_exact_moments(nlat):
    mu, w = grid.gauss_latitudes(nlat)
    assert abs(w.sum() - 2.0) < 1e-14
    for p in range(0, nlat):          # degree 2p <= 2 nlat - 1 integrates exactly
        assert abs(np.sum(w * mu ** (2 * p)) - 2.0 / (2 * p + 1)) < 2e-14
        assert abs(np.sum(w * mu ** (2 * p + 1))) < 1e-14


def test_legendre_spot_values_vs_scipy():
    mu = np.array([0.93, 0.41, -0.17, -0.88])
    P = legendre.p_tables(20, mu)
    for m in range(0, 21):
        for n in range(m, 21):
            np.testing.assert_allclose(P[m][n - m], pnm(n, m, mu), rtol=1e-12, atol=1e-13)


def test_legendre_orthonormal(g):
    for m in range(T_SMALL + 1):
        P = g.P[m][: T_SMALL + 1 - m]
        G = (P * g.w) @ P.T
        np.testing.assert_allclose(G, np.eye(T_SMALL + 1 - m), atol=2e-14)


def test_legendre_high_order_no_underflow():
    # at T255 on its 384-ring grid P_m^m underflows float64 near the poles;
    # the longdouble seed keeps the deep-evanescent values at 0 and the rest normalized
    T, nlat = 255, 384
    mu, w = grid.gauss_latitudes(nlat)
    P = legendre.p_tables(T, mu)
    for m in (0, 128, 200, 250, 255):
        Pm = P[m][: T + 1 - m]
        G = (Pm * w) @ Pm.T
        np.testing.assert_allclose(np.diag(G), 1.0, atol=5e-14)
        assert np.all(np.isfinite(Pm))


def test_h_closed_form_and_derivative():
    mu = np.linspace(-0.95, 0.95, 11)
    T = 12
    P = legendre.p_tables(T, mu)
    H = legendre.h_tables(T, mu, P)
    np.testing.assert_allclose(H[0][1], math.sqrt(1.5) * (1 - mu ** 2), atol=1e-15)
    h = 1e-5
    for m in range(T + 1):
        for n in range(m, T + 1):
            d = (pnm(n, m, mu + h) - pnm(n, m, mu - h)) / (2 * h)
            np.testing.assert_allclose(H[m][n - m], (1 - mu ** 2) * d, atol=2e-7 * max(1, n * n))


def test_single_harmonic_exact_analysis(g):
    rng = np.random.default_rng(3)
    for _ in range(12):
        m = int(rng.integers(0, T_SMALL + 1))
        n = int(rng.integers(m, T_SMALL + 1))
        spec = np.zeros(g.K, dtype=np.complex128)
        c = 1.0 if m == 0 else (0.6 - 0.8j)
        spec[sht.index(T_SMALL, m, n)] = c
        back = sht.analysis(g, sht.synthesis(g, spec))
        np.testing.assert_allclose(back, spec, atol=1e-14)


def test_band_limited_round_trip(g):
    rng = np.random.default_rng(5)
    spec = rng.standard_normal(g.K) + 1j * rng.standard_normal(g.K)
    spec[: T_SMALL + 1] = spec[: T_SMALL + 1].real
    back = sht.analysis(g, sht.synthesis(g, spec))
    np.testing.assert_allclose(back, spec, atol=5e-14)


def test_synthesis_matches_term_by_term():
    T = 6
    gg = sht.Grid(T, 12, 24)
    rng = np.random.default_rng(7)
    spec = rng.standard_normal(gg.K) + 1j * rng.standard_normal(gg.K)
    spec[: T + 1] = spec[: T + 1].real
    field = sht.synthesis(gg, spec)
    lam, phi = np.meshgrid(gg.lam, np.arcsin(gg.mu))
    np.testing.assert_allclose(field, evaluate(spec, T, lam, phi), atol=1e-12)


def test_fourier_stage_matches_direct_dft(g):
    rng = np.random.default_rng(9)
    f = rng.standard_normal((g.nlat, g.nlon))
    X = sht.fourier_analysis(g, f)
    k = np.arange(g.nlon)
    for m in (0, 1, 7, T_SMALL):
        direct = (f * np.exp(-1j * m * g.lam[None, :])).sum(axis=1) / g.nlon
        np.testing.assert_allclose(X[:, m], direct, atol=1e-14)
    assert k.size == g.nlon
