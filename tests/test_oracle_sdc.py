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


# ---------------------------------------------------------------------------
# Pins of the correction terms of one sweep (Sec. 5.1.1, eq.
# update_equation_sdcq_discrete_form).  The collocation pins above only see
# the fixed point, where every correction term vanishes; the three pins below
# constrain the terms themselves: the order gained per sweep (stated in
# Sec. 5.1.1), the explicit correction reducing to forward Euler over the
# node substeps, and the stiff-limit collapse that the LU choice of qI gives.
# The mutant tests plant plausible mistakes in copies of the oracle's
# matrices and show which pin catches each.


def _order_errors(sd, dts, kmax, lvn, A, th0):
    """One-step error after k = 1..kmax sweeps from the spread guess, against
    exp(dt A) of the probed linear-Coriolis operator; per variable, max."""
    K = lvn.K
    x0 = np.concatenate([th0.reshape(-1).real, th0.reshape(-1).imag])
    errs = np.zeros((kmax + 1, len(dts)))
    for i, dt in enumerate(dts):
        r = expm(dt * A) @ x0
        ref = (r[: 3 * K] + 1j * r[3 * K:]).reshape(3, K)
        th, fe, fi = sdc.spread(lvn, th0, sd.M + 1, True)
        for k in range(1, kmax + 1):
            th, fe, fi = sdc.sweep(lvn, sd, dt, th, fe, fi, None, True)
            errs[k, i] = max(np.abs(th[-1][v] - ref[v]).max() / np.abs(ref[v]).max() for v in range(3))
    return errs


def test_each_sweep_raises_the_order_by_one():
    """Sec. 5.1.1: each sweep raises the formal order by one until the order
    of the quadrature is reached.  From the spread guess (order 0), k sweeps
    give a one-step error O(dt^(k+1)); the slope of log(error) over log(dt)
    is fitted for k = 1..2M (3 nodes) and k = 1..6 (5 nodes; the collocation
    order 2M = 8 itself is checked by test_collocation_order_vs_expm)."""
    Tn = 6
    lvn = swe.Level(Tn, 12, 24)
    A = _probe_matrix(lvn)
    th0 = inputs.random_spectrum(Tn, 3)
    for nn, dts, kmax in ((3, (300.0, 600.0, 1200.0), 4), (5, (1000.0, 2000.0, 4000.0), 6)):
        errs = _order_errors(sdc.SDC(nn), dts, kmax, lvn, A, th0)
        slopes = [np.polyfit(np.log(dts), np.log(errs[k]), 1)[0] for k in range(1, kmax + 1)]
        for k, s in enumerate(slopes, start=1):
            assert abs(s - (k + 1)) < 0.45, (nn, k, slopes)


def _zero_history_sweep(sd, lvn, st, dt):
    """A sweep whose previous iterate has F = 0 at every node (inputs the
    sweep accepts as data): only the correction terms act."""
    nn = sd.M + 1
    th = np.repeat(st[None], nn, axis=0)
    z = np.zeros_like(th)
    return sdc.sweep(lvn, sd, dt, th, z, z.copy(), None, True)


def _euler_over_nodes(sd, lvn, st, dt):
    """Forward Euler from node 1 over the substeps dt (tau_{m+1} - tau_m)."""
    out = [st, st]
    for m in range(1, sd.M):
        h = dt * (sd.nodes[m + 1] - sd.nodes[m])
        out.append(out[-1] + h * swe.explicit_rhs(lvn, out[-1], True))
    return np.array(out)


@pytest.fixture(scope="module")
def lv_explicit_only():
    """Phibar = nu = 0 and a state with Phi = 0: F_I = 0 along the sweep,
    F_E = the linear Coriolis terms (test flag)."""
    return swe.Level(6, 12, 24, swe.Physics(phibar=0.0, nu=0.0))


@pytest.mark.parametrize("nn", [3, 5])
def test_explicit_correction_is_forward_euler_over_nodes(lv_explicit_only, nn):
    """qE is forward Euler (Sec. 5.1.1): with the previous iterate's F set to
    zero and F_I = 0, the Q-form update Theta^{m+1} = Theta^0 + dt sum_{j=1}^m
    qE_{m+1,j} F_E(Theta^j) is Euler stepping over the node substeps starting
    from Theta^1 = Theta^0 (the explicit sum starts at j = 1)."""
    sd = sdc.SDC(nn)
    st = inputs.random_spectrum(6, 5)
    st[0] = 0.0
    out, fe, fi = _zero_history_sweep(sd, lv_explicit_only, st, 500.0)
    assert np.abs(fi).max() == 0.0
    ref = _euler_over_nodes(sd, lv_explicit_only, st, 500.0)
    for i in range(nn):
        for v in (1, 2):
            assert np.abs(out[i, v] - ref[i, v]).max() <= 1e-15 * np.abs(ref[i, v]).max(), (i, v)


def _stiff_error(sd, nu, nsweeps):
    """Max over nodes 1..M and variables of the distance to the collocation
    solution after `nsweeps` sweeps from the spread guess, for F_E = 0
    (Omega = 0, linear-Coriolis flag) and a diffusion-dominated F_I."""
    Tn = 10
    lvs = swe.Level(Tn, 16, 32, swe.Physics(omega=0.0, nu=nu))
    th0 = inputs.random_spectrum(Tn, 8) + inputs.mean_geopotential(Tn)
    dt = 100.0
    th, fe, fi = sdc.spread(lvs, th0, sd.M + 1, True)
    hist = []
    for _ in range(max(nsweeps, 60)):
        th, fe, fi = sdc.sweep(lvs, sd, dt, th, fe, fi, None, True)
        hist.append(th.copy())
    ref, got = hist[-1], hist[nsweeps - 1]
    return max(np.abs(got[1:, v] - ref[1:, v]).max() / np.abs(ref[:, v]).max() for v in range(3))


@pytest.mark.parametrize("nn", [3, 5])
def test_lu_qi_collapses_in_the_stiff_limit(nn):
    """qI = U^T of the LU factorization of Q^T (Sec. 5.1.1, the choice cited
    for stiff problems): in the stiff limit the error propagation of a sweep
    tends to I - L^T, which is nilpotent, so after M sweeps the iterate
    reaches the collocation solution up to a term that vanishes as the
    stiffness grows (here dt nu n(n+1)/a^2 >= 5e3 for every n >= 1)."""
    sd = sdc.SDC(nn)
    e1 = _stiff_error(sd, 1e15, sd.M)
    e2 = _stiff_error(sd, 1e16, sd.M)
    assert e1 < 2e-4 and e2 < 0.2 * e1, (e1, e2)


def _implicit_euler_qi(sd):
    QI = np.zeros_like(sd.QI)
    for i in range(1, sd.M + 1):
        for j in range(1, i + 1):
            QI[i, j] = sd.nodes[j] - sd.nodes[j - 1]
    return QI


@pytest.mark.parametrize("nn", [3, 5])
def test_planted_sweep_mistakes_are_caught(lv_explicit_only, nn):
    """Mutants of the correction terms (planted in copies of the oracle's
    matrices) keep the collocation fixed point and the order gained per
    sweep, but fail the Euler or the stiff-limit pin."""
    st = inputs.random_spectrum(6, 5)
    st[0] = 0.0
    ref = _euler_over_nodes(sdc.SDC(nn), lv_explicit_only, st, 500.0)

    def euler_ok(sd):
        out, _, _ = _zero_history_sweep(sd, lv_explicit_only, st, 500.0)
        return all(np.abs(out[i, v] - ref[i, v]).max() <= 1e-12 * np.abs(ref[i, v]).max()
                   for i in range(nn) for v in (1, 2))

    assert euler_ok(sdc.SDC(nn))
    # qE row m used for node m+1
    mut = sdc.SDC(nn)
    QE = np.zeros_like(mut.QE)
    QE[1:] = mut.QE[:-1]
    mut.QE = QE
    assert not euler_ok(mut)
    # explicit sum over j < m instead of j <= m
    mut = sdc.SDC(nn)
    mut.QE = np.tril(mut.QE, -2)
    assert not euler_ok(mut)
    # qI: implicit Euler weights, or the LU rows shifted below the diagonal
    mut = sdc.SDC(nn)
    mut.QI = _implicit_euler_qi(mut)
    assert _stiff_error(mut, 1e15, mut.M) > 1e-2
    mut = sdc.SDC(nn)
    shifted = np.diag(np.diag(mut.QI))
    shifted[2:, 1:] += np.tril(mut.QI[1:-1, 1:], -1)
    mut.QI = shifted
    assert _stiff_error(mut, 1e15, mut.M) > 1e-2
