"""Pins of the oracle's shallow-water operators (Sec. 2, 3, 5.4).

Pins: closed forms (solid-body velocity, Laplacian eigenvalues, balanced
steady state), invariants (global means), a library solve, and brute-force
finite differences of a band-limited state evaluated term by term.
"""

import math

import numpy as np
import pytest

from oracle import sdc, sht, swe
from paper_1904_05988_amd import inputs
from tests._direct import evaluate

T, NLAT, NLON = 15, 24, 48


@pytest.fixture(scope="module")
def lv():
    return swe.Level(T, NLAT, NLON)


@pytest.fixture(scope="module")
def lv0():
    return swe.Level(T, NLAT, NLON, swe.Physics(nu=0.0))


def test_solid_body_velocity(lv):
    u0 = 20.0
    th = inputs.solid_body(T, u0)
    psi = swe.streamfunction(lv, th[1])
    chi = swe.streamfunction(lv, th[2])
    Uf, Vf = swe.uv_fourier(lv, psi, chi)
    U = sht.fourier_synthesis(lv.g, Uf)
    V = sht.fourier_synthesis(lv.g, Vf)
    np.testing.assert_allclose(U, u0 * (1 - lv.g.mu[:, None] ** 2) * np.ones_like(U), atol=1e-13)
    np.testing.assert_allclose(V, 0.0, atol=1e-13)


@pytest.mark.parametrize("m,n", [(0, 1), (0, 5), (2, 3), (4, 9), (7, 7), (3, 15)])
def test_laplacian_eigenvalues(lv, m, n):
    a = lv.phys.radius
    unit = np.zeros(lv.K, dtype=np.complex128)
    unit[sht.index(T, m, n)] = 1.0 if m == 0 else (0.3 + 0.4j)
    zero = np.zeros_like(unit)
    # chi = Y_n^m: divergence of grad chi is -n(n+1)/a^2 chi
    Uf, Vf = swe.uv_fourier(lv, zero, unit)
    div = swe._div_form(lv, Uf, Vf)
    np.testing.assert_allclose(div, -n * (n + 1) / a ** 2 * unit, atol=1e-14 * n * n / a ** 2)
    # psi = Y_n^m: curl of k x grad psi is -n(n+1)/a^2 psi
    Uf, Vf = swe.uv_fourier(lv, unit, zero)
    curl = swe._div_form(lv, Vf, -Uf)
    np.testing.assert_allclose(curl, -n * (n + 1) / a ** 2 * unit, atol=1e-14 * n * n / a ** 2)


def test_global_means_conserved(lv):
    th = inputs.seeded_state(T, 11)
    fe, fi = swe.rhs(lv, th)
    assert np.abs(fe[:, 0]).max() == 0.0 or np.abs(fe[:, 0]).max() < 1e-25
    assert np.abs(fi[:, 0]).max() == 0.0
    sd = sdc.SDC(3)
    out = sdc.serial_sdc(lv, sd, 120.0, th, nsteps=5, nsweeps=3)
    assert abs(out[0, 0] - th[0, 0]) <= 1e-15 * abs(th[0, 0])
    assert abs(out[1, 0]) < 1e-25 and abs(out[2, 0]) < 1e-25


def test_solid_body_steady_state(lv0):
    th = inputs.mean_geopotential(T) + inputs.solid_body(T, 20.0)
    fe, fi = swe.rhs(lv0, th)
    scale = np.abs(fe).max(axis=1)
    np.testing.assert_array_less(np.abs(fe + fi).max(axis=1), 1e-13 * np.maximum(scale, 1e-30) + 1e-30)
    out = sdc.serial_sdc(lv0, sdc.SDC(3), 600.0, th, nsteps=6, nsweeps=4)
    # delta is zero in this state, so its drift is measured on the zeta scale
    scales = [np.abs(th[0]).max(), np.abs(th[1]).max(), np.abs(th[1]).max()]
    for i in range(3):
        assert np.abs(out[i] - th[i]).max() <= 1e-12 * scales[i]


def test_implicit_solve_vs_linalg(lv):
    rng = np.random.default_rng(2)
    b = rng.standard_normal((3, lv.K)) + 1j * rng.standard_normal((3, lv.K))
    beta = 37.5
    x = swe.implicit_solve(lv, beta, b)
    p = lv.phys
    for k in range(0, lv.K, 7):
        lam = lv.lam[k]
        Lk = np.array([[p.nu * lam, 0, -p.phibar], [0, p.nu * lam, 0], [-lam, 0, p.nu * lam]])
        ref = np.linalg.solve(np.eye(3) - beta * Lk, b[:, k])
        np.testing.assert_allclose(x[:, k], ref, rtol=1e-13)
    # and the residual of the solved system
    blx = beta * swe.implicit_rhs(lv, x)
    res = x - blx - b
    assert np.abs(res).max() < 1e-14 * max(np.abs(blx).max(), np.abs(b).max())


def _d(f, h=1e-3):
    """4th-order central difference of a callable of one float."""
    return (f(-2 * h) - 8 * f(-h) + 8 * f(h) - f(2 * h)) / (12 * h)


def test_nonlinear_terms_vs_finite_differences():
    """N of a band-limited state (degrees <= 4, so every product stays inside
    T = 12 and is resolved exactly) against the equations of Sec. 2 evaluated
    pointwise with finite differences of the term-by-term expansion."""
    Tn = 12
    lvn = swe.Level(Tn, 20, 40)
    a, Om = lvn.phys.radius, lvn.phys.omega
    rng = np.random.default_rng(21)
    th = np.zeros((3, lvn.K), dtype=np.complex128)
    m_of, n_of = lvn.g.m_of, lvn.g.n_of
    low = (n_of <= 4) & (n_of >= 1)
    z = rng.standard_normal((3, lvn.K)) + 1j * rng.standard_normal((3, lvn.K))
    z[:, m_of == 0] = z[:, m_of == 0].real
    th[:, low] = z[:, low] * np.array([1e3, 1e-5, 3e-6])[:, None]
    th[0, 0] = math.sqrt(2) * lvn.phys.phibar
    fe = swe.explicit_rhs(lvn, th)

    psi = swe.streamfunction(lvn, th[1])
    chi = swe.streamfunction(lvn, th[2])
    phip = th[0].copy()
    phip[0] -= math.sqrt(2) * lvn.phys.phibar

    def F(spec):
        return lambda lam, phi: evaluate(spec, Tn, lam, phi)

    fpsi, fchi, fphi, fzeta = F(psi), F(chi), F(phip), F(th[1])

    def u(l, p):
        return -_d(lambda h: fpsi(l, p + h)) / a + _d(lambda h: fchi(l + h, p)) / (a * math.cos(p))

    def v(l, p):
        return _d(lambda h: fpsi(l + h, p)) / (a * math.cos(p)) + _d(lambda h: fchi(l, p + h)) / a

    def eta(l, p):
        return fzeta(l, p) + 2 * Om * math.sin(p)

    pts = [(0.3, 0.7), (2.1, -0.4), (4.0, 0.05), (5.5, -1.1), (1.2, 1.2)]
    for lam, phi in pts:
        c = math.cos(phi)
        nphi = -(_d(lambda h: fphi(lam + h, phi) * u(lam + h, phi))
                 + _d(lambda h: fphi(lam, phi + h) * v(lam, phi + h) * math.cos(phi + h))) / (a * c)
        nzeta = -(_d(lambda h: eta(lam + h, phi) * u(lam + h, phi))
                  + _d(lambda h: eta(lam, phi + h) * v(lam, phi + h) * math.cos(phi + h))) / (a * c)
        curl = (_d(lambda h: eta(lam + h, phi) * v(lam + h, phi))
                - _d(lambda h: eta(lam, phi + h) * u(lam, phi + h) * math.cos(phi + h))) / (a * c)

        def ke(l, p):
            return 0.5 * (u(l, p) ** 2 + v(l, p) ** 2)

        lap_ke = (_d(lambda h: _d(lambda k: ke(lam + h + k, phi))) / (a * c) ** 2
                  + _d(lambda h: math.cos(phi + h) * _d(lambda k: ke(lam, phi + h + k))) / (a * a * c))
        ndelta = curl - lap_ke
        got = [evaluate(fe[i], Tn, np.array(lam), np.array(phi)) for i in range(3)]
        for g_, ref, scale in zip(got, (nphi, nzeta, ndelta), np.abs(fe).max(axis=1)):
            assert abs(g_ - ref) < 2e-6 * scale * 10, (lam, phi, g_, ref)


def _mode_block(lv, k):
    """The 3 x 3 complex matrix of F_I = L at spectral slot k, probed with unit
    vectors through implicit_rhs (L acts on each mode separately)."""
    out = np.zeros((3, 3), dtype=np.complex128)
    for v in range(3):
        e = np.zeros((3, lv.K), dtype=np.complex128)
        e[v, k] = 1.0
        out[:, v] = swe.implicit_rhs(lv, e)[:, k]
    return out


@pytest.mark.parametrize("nu", [0.0, 1e5])
def test_linear_part_has_gravity_wave_frequencies(nu):
    """Sec. 2, eq. linear_wave_motion_induced_by_gravitational_forces: the
    linear part carries gravity waves, Phi'' = -Phibar n(n+1)/a^2 Phi at
    nu = 0, so the (Phi, delta) block of each mode has eigenvalues
    +-i omega_n with omega_n = sqrt(n(n+1) Phibar)/a, and zeta is stationary;
    diffusion shifts all three by nu lam_n = -nu n(n+1)/a^2."""
    lvn = swe.Level(T, NLAT, NLON, swe.Physics(nu=nu, omega=0.0))
    a, pb = lvn.phys.radius, lvn.phys.phibar
    for k in range(0, lvn.K, 5):
        n = lvn.g.n_of[k]
        w = math.sqrt(n * (n + 1) * pb) / a
        d = -nu * n * (n + 1) / a ** 2
        ev = np.linalg.eigvals(_mode_block(lvn, k))
        ev = ev[np.argsort(ev.imag)]
        ref = np.array([d - 1j * w, d + 0j, d + 1j * w])
        assert np.abs(ev - ref).max() <= 1e-12 * max(w, abs(d), 1e-30), (k, ev, ref)


def test_implicit_solve_matches_eigen_decomposition(lv):
    """(I - beta L)^{-1} b through the eigen-decomposition of each probed mode
    block: eigenvalues 1/(1 - beta mu) for mu in {nu lam_n, nu lam_n +- i omega_n}
    (the closed forms above), eigenvectors from numpy."""
    rng = np.random.default_rng(3)
    b = rng.standard_normal((3, lv.K)) + 1j * rng.standard_normal((3, lv.K))
    beta = 123.0
    x = swe.implicit_solve(lv, beta, b)
    a, pb, nu = lv.phys.radius, lv.phys.phibar, lv.phys.nu
    for k in range(1, lv.K, 11):
        n = lv.g.n_of[k]
        _, V = np.linalg.eig(_mode_block(lv, k))
        mus = np.linalg.solve(V, _mode_block(lv, k) @ V).diagonal()
        w = math.sqrt(n * (n + 1) * pb) / a
        d = -nu * n * (n + 1) / a ** 2
        closed = np.array([min((d - 1j * w, d, d + 1j * w), key=lambda z: abs(z - mu)) for mu in mus])
        ref = V @ ((np.linalg.solve(V, b[:, k])) / (1.0 - beta * closed))
        np.testing.assert_allclose(x[:, k], ref, rtol=1e-11, atol=1e-13 * np.abs(b[:, k]).max())
