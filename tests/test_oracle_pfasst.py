"""Pins of the oracle's transfers, FAS correction and PFASST (Sec. 5.1.2, 5.2, 5.3).

Pins: algebraic identities of the transfer operators (R P = I, P R a
projection, injection rows for nested Lobatto sets, exact reproduction of
quadratics), the FAS property that the restricted converged fine solution
solves the coarse problem, PFASST converging to the serial collocation
solution of all time steps, and the mailbox order of Algorithm 1.
"""

import numpy as np
import pytest

from oracle import pfasst, sdc, sht, swe, transfer
from paper_1904_05988_amd import inputs

TF, TC = 10, 5


@pytest.fixture(scope="module")
def levels():
    return swe.Level(TF, 16, 32), swe.Level(TC, 8, 18)


def test_truncate_pad_identities():
    rng = np.random.default_rng(0)
    xc = rng.standard_normal((3, 3, sht.ncoef(TC))) + 1j * rng.standard_normal((3, 3, sht.ncoef(TC)))
    xf = rng.standard_normal((5, 3, sht.ncoef(TF))) + 1j * rng.standard_normal((5, 3, sht.ncoef(TF)))
    s5, s3 = sdc.SDC(5), sdc.SDC(3)
    # R P = I on the coarse level
    np.testing.assert_allclose(transfer.restrict(s5, s3, TF, TC, transfer.interpolate(s3, s5, TC, TF, xc)), xc, atol=1e-15)
    # P R is a projection
    pr = transfer.interpolate(s3, s5, TC, TF, transfer.restrict(s5, s3, TF, TC, xf))
    pr2 = transfer.interpolate(s3, s5, TC, TF, transfer.restrict(s5, s3, TF, TC, pr))
    np.testing.assert_allclose(pr2, pr, atol=1e-14)
    # truncation keeps exactly (m, n <= Tc) at the same (m, n)
    mf, nf = sht.mn_arrays(TF)
    mc, nc = sht.mn_arrays(TC)
    t = transfer.truncate(xf[0, 0], TF, TC)
    for k in range(sht.ncoef(TC)):
        assert t[k] == xf[0, 0][sht.index(TF, mc[k], nc[k])]


@pytest.mark.parametrize("nf,nc,rows", [(5, 3, (0, 2, 4)), (3, 2, (0, 2)), (5, 2, (0, 4))])
def test_time_restriction_is_injection(nf, nc, rows):
    Pi = transfer.time_restriction(sdc.SDC(nf), sdc.SDC(nc))
    expect = np.zeros((nc, nf))
    for i, r in enumerate(rows):
        expect[i, r] = 1.0
    np.testing.assert_allclose(Pi, expect, atol=1e-14)


def test_time_interpolation_reproduces_quadratics():
    s3, s5 = sdc.SDC(3), sdc.SDC(5)
    Pi = transfer.time_interpolation(s3, s5)
    for p in range(3):
        np.testing.assert_allclose(Pi @ s3.nodes ** p, s5.nodes ** p, atol=1e-15)
    # 3 -> 5: l_0 = 2(t-1/2)(t-1), l_1 = -4t(t-1), l_2 = 2t(t-1/2)
    t = s5.nodes
    np.testing.assert_allclose(Pi, np.stack([2 * (t - .5) * (t - 1), -4 * t * (t - 1), 2 * t * (t - .5)], 1), atol=1e-15)


def test_fas_restricted_fine_solution_solves_coarse_problem(levels):
    lf, lc = levels
    s5, s3 = sdc.SDC(5), sdc.SDC(3)
    dt = 300.0
    th0 = inputs.seeded_state(TF, 12)
    th, fe, fi = sdc.spread(lf, th0, 5)
    for _ in range(40):
        th, fe, fi = sdc.sweep(lf, s5, dt, th, fe, fi)
    thc = transfer.restrict(s5, s3, TF, TC, th)
    fec = np.array([swe.explicit_rhs(lc, x) for x in thc])
    fic = np.array([swe.implicit_rhs(lc, x) for x in thc])
    tau = transfer.fas_tau(s5, s3, TF, TC, dt, fe, fi, fec, fic)
    assert np.abs(tau[0]).max() == 0.0
    # the coarse FAS residual vanishes and a coarse sweep leaves R Theta_f unchanged
    r = sdc.residual(s3, dt, thc, fec, fic, tau)
    out, _, _ = sdc.sweep(lc, s3, dt, thc, fec, fic, tau)
    for v in range(3):
        scale = np.abs(thc[:, v]).max()
        assert np.abs(r[:, v]).max() <= 1e-13 * scale
        assert np.abs(out[:, v] - thc[:, v]).max() <= 1e-13 * scale
    # without tau the coarse sweep does move it (the correction is doing work)
    out0, _, _ = sdc.sweep(lc, s3, dt, thc, fec, fic, None)
    assert np.abs(out0[-1, 1] - thc[-1, 1]).max() > 1e-9 * np.abs(thc[:, 1]).max()


def test_mailbox_order_is_checked():
    mb = pfasst.Mailbox()
    with pytest.raises(RuntimeError):
        mb.recv(("fine", 0, 1))
    mb.send(("fine", 0, 1), np.zeros(2))
    mb.recv(("fine", 0, 1))
    with pytest.raises(RuntimeError):
        mb.send(("fine", 0, 1), np.zeros(2))


def _serial_collocation(lv, sd, dt, th0, nsteps, nsweeps=40):
    out = []
    x = th0
    for _ in range(nsteps):
        th, fe, fi = sdc.spread(lv, x, sd.M + 1)
        for _ in range(nsweeps):
            th, fe, fi = sdc.sweep(lv, sd, dt, th, fe, fi)
        out.append(th[-1])
        x = th[-1]
    return np.array(out)


@pytest.mark.slow
def test_pfasst_converges_to_serial_collocation(levels):
    lf, lc = levels
    s5, s3 = sdc.SDC(5), sdc.SDC(3)
    dt, nts = 300.0, 4
    th0 = inputs.seeded_state(TF, 13)
    ref = _serial_collocation(lf, s5, dt, th0, nts)
    res = pfasst.run(lf, lc, s5, s3, dt, th0, nts, 25)
    errs = [max(np.abs(ev[:, v] - ref[:, v]).max() / np.abs(ref[:, v]).max() for v in range(3))
            for ev in res.end_values]
    assert errs[-1] < 1e-12, errs
    assert errs[0] > 1e-9            # it really iterated towards the fixed point
    assert errs[-1] < errs[2] < errs[0]


def test_pfasst_single_slice_is_two_level_iteration(levels):
    lf, lc = levels
    s5, s3 = sdc.SDC(5), sdc.SDC(3)
    th0 = inputs.seeded_state(TF, 14)
    ref = _serial_collocation(lf, s5, 300.0, th0, 1)
    res = pfasst.run(lf, lc, s5, s3, 300.0, th0, 1, 12)
    for v in range(3):
        assert np.abs(res.end_values[-1][0, v] - ref[0, v]).max() <= 1e-12 * np.abs(ref[0, v]).max()


def test_residual_stop_equals_fixed_iterations(levels):
    """The convergence check (future work of Sec. 5.2.2, reading: stop after
    the fine sweep of the first iteration whose fine collocation residuals are
    at most tol for every time step and variable) stops where the residual
    history first falls below tol, with the state of the fixed-iteration run
    of that many iterations, bit for bit; without tol all iterations run."""
    lf, lc = levels
    sf, sc = sdc.SDC(5), sdc.SDC(3)
    th0 = inputs.seeded_state(TF, 21)
    full = pfasst.run(lf, lc, sf, sc, 200.0, th0, 4, 8)
    assert full.iterations == 8 and len(full.residuals) == 8
    hist = np.array([r.max(axis=0) for r in full.residuals])       # [iteration, var]
    for v in range(3):
        assert hist[-1, v] < 1e-3 * hist[0, v], hist[:, v]           # the iteration converges
    tol = hist[3] * 1.01                       # met by the 4th iteration's residuals (or earlier)
    first = next(i for i in range(8) if np.all(hist[i] <= tol)) + 1
    assert first <= 4
    stopped = pfasst.run(lf, lc, sf, sc, 200.0, th0, 4, 8, tol=tol)
    assert stopped.iterations == first
    fixed = pfasst.run(lf, lc, sf, sc, 200.0, th0, 4, first)
    np.testing.assert_array_equal(stopped.end_values[-1], fixed.end_values[-1])
    np.testing.assert_array_equal(np.array(stopped.theta), np.array(fixed.theta))
