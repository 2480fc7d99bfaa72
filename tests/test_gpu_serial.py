"""GPU parity of the serial comparators of Sec. 5.5 on the library's kernels:
SDC(M+1, N_S) time stepping (pfsh_sdc_run) and MLSDC(Mf+1, Mc+1, N_ML, alpha)
(pfsh_mlsdc_run) against the oracle, over several steps, on the batched and
the fused small-batch sweep paths."""

import numpy as np
import pytest

from oracle import mlsdc, sdc, swe
from paper_1904_05988_amd import pfsh
from tests._gpu import level_pair, rel_err, seeded, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nn,B,nsweeps", [(3, 2, 2), (5, 3, 3), (5, 1, 4)])
def test_sdc_run_matches_oracle(nn, B, nsweeps):
    T, nlat, nlon, dt, nsteps = 31, 48, 96, 150.0, 3
    gl, ol = level_pair(T, nlat, nlon, nn, max_batch=B)
    states = seeded(T, range(370, 370 + B))
    th, fe, fi = gl.space_time(B), gl.space_time(B), gl.space_time(B)
    th[:, 0] = to_dev(states)
    gl.sdc_run(dt, th, fe, fi, nsteps, nsweeps)
    got = to_host(th)
    for b in range(B):
        ref = sdc.serial_sdc(ol, sdc.SDC(nn), dt, states[b], nsteps, nsweeps)
        assert np.all(rel_err(got[b, 0], ref) <= 1e-11), b
        assert np.array_equal(got[b, 0], got[b, -1])


@pytest.mark.parametrize("members,n_iter", [(1, 3), (2, 2)])
def test_mlsdc_run_matches_oracle(members, n_iter):
    Tf, Tc, nf, nc, dt, nsteps = 15, 7, 5, 3, 300.0, 2
    gf = pfsh.Level(Tf, 24, 48, nf, max_batch=members)
    gc = pfsh.Level(Tc, 12, 24, nc, max_batch=members)
    of, oc = swe.Level(Tf, 24, 48), swe.Level(Tc, 12, 24)
    states = seeded(Tf, range(380, 380 + members))
    pf = pfsh.Pfasst(gf, gc, 1, members)
    th, fe, fi = gf.space_time(members), gf.space_time(members), gf.space_time(members)
    th[:, 0] = to_dev(states)
    pf.mlsdc_run(dt, th, fe, fi, nsteps, n_iter)
    got = to_host(th)
    for b in range(members):
        ref = mlsdc.run(of, oc, sdc.SDC(nf), sdc.SDC(nc), dt, states[b], nsteps, n_iter)
        assert np.all(rel_err(got[b, 0], ref[-1]) <= 1e-11), b
    pf.close()
    pf2 = pfsh.Pfasst(pfsh.Level(Tf, 24, 48, nf, max_batch=2), pfsh.Level(Tc, 12, 24, nc, max_batch=2), 2)
    with pytest.raises(pfsh.PfshError):
        pf2.mlsdc_run(dt, *(pf2.fine.space_time(2) for _ in range(3)), 1, 1)
    pf2.close()
