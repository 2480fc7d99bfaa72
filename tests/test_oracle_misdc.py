"""Pins of the oracle's two-substep implicit step (Sec. 5.1.1, last paragraph:
the implementation splits the implicit step into a substep in the physical
linear terms and a substep in the artificial diffusion, the multi-implicit
SDC of the cited Bourlioux, Layton and Minion work).

Pins: each substep solves its own operator, whose eigenvalues are closed forms
(gravity waves +-i sqrt(n(n+1) Phibar)/a, diffusion nu lam_n); without
diffusion the split sweep is the combined sweep bit for bit; with diffusion
one split sweep differs from the combined one, yet the iteration converges to
the same collocation solution; each split sweep raises the order by one
(against expm of the probed operator); a planted mistake (the old diffusion
value left out of both substeps) moves the fixed point and is caught."""

import math

import numpy as np
import pytest
from scipy.linalg import expm

from oracle import sdc, swe
from paper_1904_05988_amd import inputs

T, NLAT, NLON = 10, 16, 32


@pytest.fixture(scope="module")
def lv():
    return swe.Level(T, NLAT, NLON)


def _block(f, lv, k):
    out = np.zeros((3, 3), dtype=np.complex128)
    for v in range(3):
        e = np.zeros((3, lv.K), dtype=np.complex128)
        e[v, k] = 1.0
        out[:, v] = f(lv, e)[:, k]
    return out


def test_substep_operators_and_solves(lv):
    a, pb, nu = lv.phys.radius, lv.phys.phibar, lv.phys.nu
    beta = 37.0
    rng = np.random.default_rng(1)
    b = rng.standard_normal((3, lv.K)) + 1j * rng.standard_normal((3, lv.K))
    for k in range(1, lv.K, 7):
        n = lv.g.n_of[k]
        ev = np.linalg.eigvals(_block(swe.gravity_rhs, lv, k))
        ev = ev[np.argsort(ev.imag)]
        w = math.sqrt(n * (n + 1) * pb) / a
        np.testing.assert_allclose(ev, [-1j * w, 0.0, 1j * w], atol=1e-12 * w)
        np.testing.assert_allclose(np.linalg.eigvals(_block(swe.diffusion_rhs, lv, k)),
                                   [-nu * n * (n + 1) / a ** 2] * 3, rtol=1e-14)
    for solve, op in ((swe.gravity_solve, swe.gravity_rhs), (swe.diffusion_solve, swe.diffusion_rhs)):
        x = solve(lv, beta, b)
        t = beta * op(lv, x)
        scale = max(np.abs(b).max(), np.abs(x).max(), np.abs(t).max())
        assert np.abs(x - t - b).max() <= 1e-14 * scale


def _spread_sweeps(lv, sd, dt, th0, n, misdc, lin=False):
    th, fe, fi = sdc.spread(lv, th0, sd.M + 1, lin)
    for _ in range(n):
        th, fe, fi = sdc.sweep(lv, sd, dt, th, fe, fi, None, lin, misdc)
    return th, fe, fi


@pytest.mark.parametrize("nn", [3, 5])
def test_split_equals_combined_without_diffusion(nn):
    lv0 = swe.Level(T, NLAT, NLON, swe.Physics(nu=0.0))
    sd = sdc.SDC(nn)
    th0 = inputs.seeded_state(T, 11)
    a = _spread_sweeps(lv0, sd, 300.0, th0, 2, False)
    b = _spread_sweeps(lv0, sd, 300.0, th0, 2, True)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("nn", [3, 5])
def test_split_has_the_same_collocation_fixed_point(lv, nn):
    sd = sdc.SDC(nn)
    dt = 600.0
    th0 = inputs.seeded_state(T, 12)
    one_c = _spread_sweeps(lv, sd, dt, th0, 1, False)[0]
    one_s = _spread_sweeps(lv, sd, dt, th0, 1, True)[0]
    scale = np.abs(one_c[-1]).max(axis=1)
    scale[0] = np.abs(one_c[-1][0, 1:]).max()
    d1 = np.abs(one_s[-1] - one_c[-1]).max(axis=1) / scale
    assert d1.max() > 1e-10, d1            # the split acts on one sweep
    th_c, fe_c, fi_c = _spread_sweeps(lv, sd, dt, th0, 40, False)
    th_s, fe_s, fi_s = _spread_sweeps(lv, sd, dt, th0, 40, True)
    r = sdc.residual_norm(sd, dt, th_s, fe_s, fi_s)
    assert np.all(r <= 1e-13 * np.abs(th_s).max(axis=(0, 2))), r
    d = np.abs(th_s - th_c).max(axis=(0, 2)) / np.abs(th_c).max(axis=(0, 2))
    assert np.all(d <= 1e-12), d


def test_split_sweep_raises_the_order_by_one():
    """The order gained per sweep (Sec. 5.1.1) holds for the split implicit
    step: one-step errors after k sweeps from the spread guess, against
    exp(dt A) of the probed linear-Coriolis operator with diffusion on."""
    Tn = 6
    lvn = swe.Level(Tn, 12, 24)
    K = lvn.K
    n = 6 * K
    A = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        th = (e[: 3 * K] + 1j * e[3 * K:]).reshape(3, K)
        fe, fi = swe.rhs(lvn, th, linear_coriolis=True)
        f = (fe + fi).reshape(-1)
        A[:, i] = np.concatenate([f.real, f.imag])
    th0 = inputs.random_spectrum(Tn, 3)
    x0 = np.concatenate([th0.reshape(-1).real, th0.reshape(-1).imag])
    sd = sdc.SDC(3)
    dts = (300.0, 600.0, 1200.0)
    errs = np.zeros((5, len(dts)))
    for i, dt in enumerate(dts):
        r = expm(dt * A) @ x0
        ref = (r[: 3 * K] + 1j * r[3 * K:]).reshape(3, K)
        th, fe, fi = sdc.spread(lvn, th0, 3, True)
        for k in range(1, 5):
            th, fe, fi = sdc.sweep(lvn, sd, dt, th, fe, fi, None, True, True)
            errs[k, i] = max(np.abs(th[-1][v] - ref[v]).max() / np.abs(ref[v]).max() for v in range(3))
    slopes = [np.polyfit(np.log(dts), np.log(errs[k]), 1)[0] for k in range(1, 5)]
    for k, s in enumerate(slopes, start=1):
        assert abs(s - (k + 1)) < 0.45, slopes


def test_planted_mistake_moves_the_fixed_point(lv, monkeypatch):
    """Leaving the old diffusion value out of both substeps (L2 Theta^(k)
    taken as 0 inside the split) turns the node equation into
    (I - beta L2)(I - beta L1) Theta = b: the converged iterate is no longer
    the collocation solution."""
    sd = sdc.SDC(3)
    dt = 600.0
    th0 = inputs.seeded_state(T, 12)
    monkeypatch.setattr(sdc.swe, "diffusion_rhs", lambda lv_, th: np.zeros_like(th))
    th, fe, fi = _spread_sweeps(lv, sd, dt, th0, 40, True)
    r = sdc.residual_norm(sd, dt, th, fe, fi)
    assert np.any(r > 1e-9 * np.abs(th).max(axis=(0, 2))), r
