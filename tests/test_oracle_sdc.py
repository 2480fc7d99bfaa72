"""Pins of the oracle's SDC matrices, sweep and collocation fixed point (Sec. 5.1.1).

Pins: closed-form node sets and integration weights, the LU property of qI,
the collocation fixed point, the diagonal Pade approximant of exp that the
Lobatto collocation reproduces on a linear problem, the collocation order
against scipy.linalg.expm of a probed operator, and independence of the
converged result from the choice of qI.
"""

import math

import numpy as np
import pytest
from scipy.linalg import expm

from oracle import sdc, swe
from paper_1904_05988_amd import inputs


def test_lobatto_nodes_closed_form():
    np.testing.assert_allclose(sdc.lobatto_nodes(2), [0, 1], atol=1e-16)
    np.testing.assert_allclose(sdc.lobatto_nodes(3), [0, 0.5, 1], atol=1e-16)
    r = math.sqrt(3.0 / 7.0)
    np.testing.assert_allclose(sdc.lobatto_nodes(5), [0, (1 - r) / 2, 0.5, (1 + r) / 2, 1], atol=1e-15)


def test_q_matrix_closed_forms():
    s3 = sdc.SDC(3)
    np.testing.assert_allclose(s3.Q, [[0, 0, 0], [5 / 24, 1 / 3, -1 / 24], [1 / 6, 2 / 3, 1 / 6]], atol=1e-15)
    np.testing.assert_allclose(s3.QI, [[0, 0, 0], [0, 1 / 3, 0], [0, 2 / 3, 1 / 4]], atol=1e-15)
    np.testing.assert_allclose(s3.QE, [[0, 0, 0], [0.5, 0, 0], [0.5, 0.5, 0]], atol=1e-16)
    s5 = sdc.SDC(5)
    np.testing.assert_allclose(s5.Q[-1], [1 / 20, 49 / 180, 16 / 45, 49 / 180, 1 / 20], atol=1e-15)
    np.testing.assert_allclose(np.diag(s5.QI)[1:], [0.1197448, 0.2328109, 0.2348679, 1 / 11], atol=1e-7)
    np.testing.assert_allclose(np.diag(s5.QI)[-1], 1 / 11, atol=1e-14)


@pytest.mark.parametrize("nn", [2, 3, 5])
def test_q_integrates_polynomials_exactly(nn):
    s = sdc.SDC(nn)
    for p in range(nn):
        np.testing.assert_allclose(s.Q @ s.nodes ** p, s.nodes ** (p + 1) / (p + 1), atol=1e-15)


@pytest.mark.parametrize("nn", [3, 5])
def test_qi_is_transposed_u_factor(nn):
    s = sdc.SDC(nn)
    U = s.QI[1:, 1:].T
    assert np.allclose(np.tril(U, -1), 0)
    L = s.Q[1:, 1:].T @ np.linalg.inv(U)
    np.testing.assert_allclose(np.diag(L), 1.0, atol=1e-14)
    assert np.allclose(np.triu(L, 1), 0, atol=1e-14)
    assert np.all(s.QI[:, 0] == 0) and np.all(s.QI[0] == 0)


T, NLAT, NLON = 10, 16, 32


@pytest.fixture(scope="module")
def lv():
    return swe.Level(T, NLAT, NLON)


def _converge(lv, sd, dt, th0, nsweeps, lin=False):
    th, fe, fi = sdc.spread(lv, th0, sd.M + 1, lin)
    for _ in range(nsweeps):
        th, fe, fi = sdc.sweep(lv, sd, dt, th, fe, fi, None, lin)
    return th, fe, fi


def test_fixed_point_is_collocation(lv):
    sd = sdc.SDC(5)
    th0 = inputs.seeded_state(T, 4)
    th, fe, fi = _converge(lv, sd, 120.0, th0, 30)
    r = sdc.residual_norm(sd, 120.0, th, fe, fi)
    scale = np.abs(th).max(axis=(0, 2))
    assert np.all(r <= 1e-13 * scale), r / scale


def _pade_num(z, nn):
    if nn == 3:
        return [1, 1 / 2, 1 / 12]
    return [1, 1 / 2, 3 / 28, 1 / 84, 1 / 1680]


def _matpoly(c, A):
    out = np.zeros_like(A)
    P = np.eye(A.shape[0], dtype=A.dtype)
    for ck in c:
        out = out + ck * P
        P = P @ A
    return out


@pytest.mark.parametrize("nn", [3, 5])
def test_linear_converged_equals_diagonal_pade(nn):
    """Omega = 0 and the linear-Coriolis test flag make F_E = 0: the converged
    Lobatto collocation end value is R(dt A) Theta^0 with R = p(z)/p(-z)."""
    lv0 = swe.Level(T, NLAT, NLON, swe.Physics(omega=0.0))
    sd = sdc.SDC(nn)
    dt = 900.0
    th0 = inputs.random_spectrum(T, 8) + inputs.mean_geopotential(T)
    th, _, _ = _converge(lv0, sd, dt, th0, 40, lin=True)
    c = _pade_num(None, nn)
    p = lv0.phys
    scale = np.abs(th0).max(axis=1)
    for k in range(lv0.K):
        lam = lv0.lam[k]
        A = np.array([[p.nu * lam, 0, -p.phibar], [0, p.nu * lam, 0], [-lam, 0, p.nu * lam]])
        R = _matpoly(c, dt * A) @ np.linalg.inv(_matpoly(c, -dt * A))
        ref = R @ th0[:, k]
        assert np.all(np.abs(th[-1][:, k] - ref) <= 1e-12 * np.abs(ref) + 1e-13 * scale), k


def _probe_matrix(lv):
    """Real matrix of Theta -> F_E + F_I with the linear-Coriolis flag."""
    K = lv.K
    n = 6 * K
    A = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        th = (e[: 3 * K] + 1j * e[3 * K:]).reshape(3, K)
        fe, fi = swe.rhs(lv, th, linear_coriolis=True)
        f = (fe + fi).reshape(-1)
        A[:, i] = np.concatenate([f.real, f.imag])
    return A


@pytest.mark.slow
def test_collocation_order_vs_expm():
    """With enough sweeps, SDC on M+1 Lobatto nodes reaches the collocation
    solution, whose one-step error against exp(dt A) behaves like dt^(2M+1)
    (global order 2M).  The slope of log(error) over log(dt) is fitted."""
    Tn = 6
    lvn = swe.Level(Tn, 12, 24)
    A = _probe_matrix(lvn)
    th0 = inputs.random_spectrum(Tn, 3)
    x0 = np.concatenate([th0.reshape(-1).real, th0.reshape(-1).imag])
    for nn, dts, lo, hi in ((3, (1000.0, 500.0, 250.0), 4.6, 5.8),
                            (5, (3000.0, 4500.0, 6000.0, 9000.0), 7.3, 10.5)):
        sd = sdc.SDC(nn)
        errs = []
        for dt in dts:
            th, _, _ = _converge(lvn, sd, dt, th0, 100, lin=True)
            x = np.concatenate([th[-1].reshape(-1).real, th[-1].reshape(-1).imag])
            ref = expm(dt * A) @ x0
            errs.append(np.abs(x - ref).max() / np.abs(ref).max())
        slope = np.polyfit(np.log(dts), np.log(errs), 1)[0]
        assert lo < slope < hi, (nn, errs, slope)


def test_converged_result_independent_of_qi(lv):
    sd = sdc.SDC(3)
    th0 = inputs.seeded_state(T, 6)
    a, _, _ = _converge(lv, sd, 120.0, th0, 30)
    be = sdc.SDC(3)
    QI = np.zeros_like(be.QI)
    for i in range(1, 3):
        for j in range(1, i + 1):
            QI[i, j] = be.nodes[j] - be.nodes[j - 1]      # implicit Euler
    be.QI = QI
    b, _, _ = _converge(lv, be, 120.0, th0, 60)
    for v in range(3):
        assert np.abs(a[-1][v] - b[-1][v]).max() <= 1e-12 * np.abs(a[-1][v]).max()
