"""GPU parity at even truncations and at coarsening ratios other than 1/2.

With T even, T+1 orders is odd: in the batched sweep-node kernel every order m
pairs with T+1-m (no order stands alone but order 0), and the parity split of
an order has one even-parity degree more than with T odd.  Sec. 5.3 allows any
coarsening ratio alpha = (T_c+1)/(T_f+1); here T31 -> T20, T30 -> T14 and a
PFASST block T30 / T12 (alpha = 13/31) are checked against the oracle, element
by element, with the batched (3 slices) and the fused small-batch (1 slice)
sweep paths."""

import numpy as np
import pytest

from oracle import pfasst as opf
from oracle import sdc, sht, swe, transfer
from paper_1904_05988_amd import pfsh
from tests._gpu import level_pair, oracle_spread_batch, rel_err, seeded, to_dev, to_host

pytestmark = pytest.mark.gpu

EVEN = [(14, 24, 48), (30, 48, 96)]


@pytest.mark.parametrize("T,nlat,nlon", EVEN)
def test_transforms_at_even_truncation(T, nlat, nlon):
    gl, ol = level_pair(T, nlat, nlon, 3, max_batch=2)
    rng = np.random.default_rng(300 + T)
    spec = rng.standard_normal((5, gl.K)) + 1j * rng.standard_normal((5, gl.K))
    spec[:, : T + 1] = spec[:, : T + 1].real
    grid = to_host(gl.sh_synthesis(to_dev(spec)))
    for f in range(5):
        ref = sht.synthesis(ol.g, spec[f])
        assert np.abs(grid[f] - ref).max() <= 1e-13 * np.abs(ref).max(), f
    g = rng.standard_normal((6, nlat, nlon))
    back = to_host(gl.sh_analysis(to_dev(g)))
    for f in range(6):
        ref = sht.analysis(ol.g, g[f])
        assert np.abs(back[f] - ref).max() <= 1e-13 * np.abs(ref).max(), f
    rt = to_host(gl.sh_analysis(gl.sh_synthesis(to_dev(spec))))
    assert np.abs(rt - spec).max() <= 1e-13 * np.abs(spec).max()


@pytest.mark.parametrize("T,nlat,nlon", EVEN)
def test_rhs_at_even_truncation(T, nlat, nlon):
    B = 3
    gl, ol = level_pair(T, nlat, nlon, 3, max_batch=B)
    states = seeded(T, range(310, 310 + B))
    fe, fi = gl.rhs(to_dev(states))
    fe, fi = to_host(fe), to_host(fi)
    for b in range(B):
        rfe, rfi = swe.rhs(ol, states[b])
        assert np.all(rel_err(fe[b], rfe) <= 1e-12), b
        assert np.all(rel_err(fi[b], rfi) <= 1e-13), b


@pytest.mark.parametrize("T,nlat,nlon", EVEN)
@pytest.mark.parametrize("nn,B", [(3, 3), (5, 3), (3, 1), (5, 1)])
def test_sweeps_at_even_truncation(T, nlat, nlon, nn, B):
    """Batch 3 takes the separate kernels (paired orders), batch 1 the fused
    per-order node; two sweeps from the spread guess, every node."""
    dt = 150.0
    gl, ol = level_pair(T, nlat, nlon, nn, max_batch=B)
    states = seeded(T, range(320, 320 + B))
    th, fe, fi = gl.space_time(B), gl.space_time(B), gl.space_time(B)
    e, i = gl.rhs(to_dev(states))
    th[:, 0] = to_dev(states)
    fe[:, 0] = e
    fi[:, 0] = i
    gl.spread(th, fe, fi)
    rth, rfe, rfi = oracle_spread_batch(ol, states, nn)
    sd = sdc.SDC(nn)
    for sweep in range(2):
        gl.sdc_sweep(dt, th, fe, fi)
        for b in range(B):
            rth[b], rfe[b], rfi[b] = sdc.sweep(ol, sd, dt, rth[b], rfe[b], rfi[b])
        gth, gfe, gfi = to_host(th), to_host(fe), to_host(fi)
        for b in range(B):
            for n in range(nn):
                assert np.all(rel_err(gth[b, n], rth[b, n]) <= 1e-12), (sweep, b, n)
                assert np.all(rel_err(gfe[b, n], rfe[b, n]) <= 1e-11), (sweep, b, n)
                assert np.all(rel_err(gfi[b, n], rfi[b, n]) <= 1e-12), (sweep, b, n)


@pytest.mark.parametrize("Tf,gf_grid,Tc,gc_grid", [(31, (48, 96), 20, (32, 64)),
                                                   (30, (48, 96), 14, (24, 48)),
                                                   (30, (48, 96), 12, (24, 48))])
def test_transfers_at_other_coarsening_ratios(Tf, gf_grid, Tc, gc_grid):
    nf, nc, B = 5, 3, 2
    gf, _ = level_pair(Tf, *gf_grid, nf, max_batch=B)
    gc, _ = level_pair(Tc, *gc_grid, nc, max_batch=B)
    sf, sc = sdc.SDC(nf), sdc.SDC(nc)
    rng = np.random.default_rng(Tf * 100 + Tc)
    xf = rng.standard_normal((B, nf, 3, gf.K)) + 1j * rng.standard_normal((B, nf, 3, gf.K))
    xn = rng.standard_normal((B, nc, 3, gc.K)) + 1j * rng.standard_normal((B, nc, 3, gc.K))
    xo = rng.standard_normal((B, nc, 3, gc.K)) + 1j * rng.standard_normal((B, nc, 3, gc.K))
    r = to_host(pfsh.restrict(gf, gc, to_dev(xf)))
    for b in range(B):
        np.testing.assert_allclose(r[b], transfer.restrict(sf, sc, Tf, Tc, xf[b]), rtol=0, atol=1e-13)
    io = to_dev(xf.copy())
    pfsh.interpolate_add(gc, gf, to_dev(xn), to_dev(xo), io)
    io = to_host(io)
    for b in range(B):
        ref = xf[b] + transfer.interpolate(sc, sf, Tc, Tf, xn[b] - xo[b])
        np.testing.assert_allclose(io[b], ref, rtol=0, atol=1e-13)
    tau = to_host(pfsh.fas_tau(gf, gc, 90.0, to_dev(xf * 1e-9), to_dev(xf[:, ::-1].copy() * 1e-9),
                               to_dev(xn * 1e-9), to_dev(xo * 1e-9)))
    for b in range(B):
        ref = transfer.fas_tau(sf, sc, Tf, Tc, 90.0, xf[b] * 1e-9, xf[b, ::-1] * 1e-9,
                               xn[b] * 1e-9, xo[b] * 1e-9)
        np.testing.assert_allclose(tau[b], ref, rtol=0, atol=1e-20)


def test_pfasst_even_truncation_and_coarsening_13_31():
    """PFASST(4, 5, 3, 3) with fine T30 on 48 x 96 and coarse T12 on 24 x 48:
    the predictor and every node after each iteration against the oracle (the
    coarse chain runs the fused per-order node at batch 1)."""
    Tf, Tc, nf, nc, dt, n_ts, n_iter = 30, 12, 5, 3, 150.0, 4, 3
    gf = pfsh.Level(Tf, 48, 96, nf, max_batch=n_ts)
    gc = pfsh.Level(Tc, 24, 48, nc, max_batch=n_ts)
    of, oc = swe.Level(Tf, 48, 96), swe.Level(Tc, 24, 48)
    th0 = seeded(Tf, (330,))[0]
    ref = opf.run(of, oc, sdc.SDC(nf), sdc.SDC(nc), dt, th0, n_ts, n_iter)
    pf = pfsh.Pfasst(gf, gc, n_ts)
    thf, fef, fif = gf.space_time(n_ts), gf.space_time(n_ts), gf.space_time(n_ts)
    pf.predict(dt, to_dev(th0[None]), thf, fef, fif)
    got = to_host(thf)[:, -1]
    for n in range(n_ts):
        assert np.all(rel_err(got[n], ref.pred_end[n]) <= 1e-12), ("pred", n)
    for k in range(n_iter):
        last = k == n_iter - 1
        pf.iterate(dt, thf, fef, fif, last=last)
        got = to_host(thf)
        for n in range(n_ts):
            if last:
                assert np.all(rel_err(got[n, -1], ref.end_values[k][n]) <= 1e-11), (k, n)
            else:
                for i in range(nf):
                    assert np.all(rel_err(got[n, i], ref.after_iter[k][n, i]) <= 1e-11), (k, n, i)
    pf.close()
