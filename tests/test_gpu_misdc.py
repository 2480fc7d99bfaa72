"""GPU parity of the two-substep implicit step (Sec. 5.1.1, last paragraph: a
substep in the physical linear terms, then one in the artificial diffusion)
against the oracle's split sweep, on the batched (paired-order) and the fused
small-batch sweep paths, and inside a PFASST block."""

import numpy as np
import pytest

from oracle import pfasst as opf
from oracle import sdc, swe
from paper_1904_05988_amd import pfsh
from tests._gpu import level_pair, oracle_spread_batch, rel_err, seeded, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("T,nlat,nlon", [(31, 48, 96), (30, 48, 96)])
@pytest.mark.parametrize("nn,B", [(3, 1), (3, 3), (5, 2), (5, 3)])
def test_split_sweeps_match_oracle(T, nlat, nlon, nn, B):
    dt = 300.0
    gl, ol = level_pair(T, nlat, nlon, nn, max_batch=B)
    gl.set_implicit("split")
    states = seeded(T, range(340, 340 + B))
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
            rth[b], rfe[b], rfi[b] = sdc.sweep(ol, sd, dt, rth[b], rfe[b], rfi[b], None, False, True)
        gth, gfe, gfi = to_host(th), to_host(fe), to_host(fi)
        for b in range(B):
            for n in range(nn):
                assert np.all(rel_err(gth[b, n], rth[b, n]) <= 1e-12), (sweep, b, n)
                assert np.all(rel_err(gfe[b, n], rfe[b, n]) <= 1e-11), (sweep, b, n)
                assert np.all(rel_err(gfi[b, n], rfi[b, n]) <= 1e-12), (sweep, b, n)
    # the split is active: one combined sweep from the same start differs
    gc, _ = level_pair(T, nlat, nlon, nn, max_batch=B)
    tc, ec, ic = gc.space_time(B), gc.space_time(B), gc.space_time(B)
    e, i = gc.rhs(to_dev(states))
    tc[:, 0] = to_dev(states)
    ec[:, 0] = e
    ic[:, 0] = i
    gc.spread(tc, ec, ic)
    gc.sdc_sweep(dt, tc, ec, ic)
    gc.sdc_sweep(dt, tc, ec, ic)
    assert np.max(rel_err(to_host(tc)[0, -1], gth[0, -1])) > 1e-10


def test_split_pfasst_matches_oracle():
    Tf, Tc, nf, nc, dt, n_ts, n_iter = 15, 7, 5, 3, 300.0, 4, 3
    gf = pfsh.Level(Tf, 24, 48, nf, max_batch=n_ts)
    gc = pfsh.Level(Tc, 12, 24, nc, max_batch=n_ts)
    gf.set_implicit("split")
    gc.set_implicit("split")
    of, oc = swe.Level(Tf, 24, 48), swe.Level(Tc, 12, 24)
    th0 = seeded(Tf, (350,))[0]
    ref = opf.run(of, oc, sdc.SDC(nf), sdc.SDC(nc), dt, th0, n_ts, n_iter, misdc=True)
    pf = pfsh.Pfasst(gf, gc, n_ts)
    thf, fef, fif = gf.space_time(n_ts), gf.space_time(n_ts), gf.space_time(n_ts)
    pf.predict(dt, to_dev(th0[None]), thf, fef, fif)
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
    assert pfsh.lib().pfsh_level_set_implicit(gf.handle, 7) == -1      # PFSH_EINVAL
