"""GPU parity of the one-device PFASST block (Sec. 5.2) against the oracle's
mailbox PFASST: predictor and every iteration's fine last-node values, and
convergence to the serial collocation solution."""

import numpy as np
import pytest

from oracle import pfasst as opf
from oracle import sdc, swe
from paper_1904_05988_amd import pfsh
from tests._gpu import DEV, rel_err, seeded, to_dev, to_host

pytestmark = pytest.mark.gpu


def _levels(Tf, Tc, nf, nc, B, gf_grid, gc_grid, precision="fp64"):
    gf = pfsh.Level(Tf, *gf_grid, nf, max_batch=B, precision=precision)
    gc = pfsh.Level(Tc, *gc_grid, nc, max_batch=B, precision=precision)
    of = swe.Level(Tf, *gf_grid)
    oc = swe.Level(Tc, *gc_grid)
    return gf, gc, of, oc


@pytest.mark.parametrize("n_ts,n_iter", [(4, 4), (1, 3), (3, 2)])
def test_pfasst_iterations_match_oracle(n_ts, n_iter):
    Tf, Tc, nf, nc, dt = 15, 7, 5, 3, 300.0
    gf, gc, of, oc = _levels(Tf, Tc, nf, nc, n_ts, (24, 48), (12, 24))
    th0 = seeded(Tf, (50,))[0]
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
            if last:          # the last iteration stops after the fine sweep
                e = rel_err(got[n, -1], ref.end_values[k][n])
                assert np.all(e <= 1e-11), (k, n, e)
            else:             # full iteration A-D: compare every fine node
                for i in range(nf):
                    e = rel_err(got[n, i], ref.after_iter[k][n, i])
                    assert np.all(e <= 1e-11), (k, n, i, e)
    # the full fine solution after the last iteration
    full = to_host(thf)
    for n in range(n_ts):
        for i in range(nf):
            assert np.all(rel_err(full[n, i], ref.theta[n][i]) <= 1e-11)


def test_pfasst_members_match_oracle_per_member():
    """Ensemble members share the batch but not their arithmetic: each member
    follows the oracle's PFASST of its own initial condition."""
    Tf, Tc, nf, nc, dt, n_ts, M, n_iter = 15, 7, 5, 3, 300.0, 3, 2, 4
    gf, gc, of, oc = _levels(Tf, Tc, nf, nc, n_ts * M, (24, 48), (12, 24))
    th0 = seeded(Tf, (60, 61))
    pf = pfsh.Pfasst(gf, gc, n_ts, members=M)
    B = n_ts * M
    thf, fef, fif = gf.space_time(B), gf.space_time(B), gf.space_time(B)
    pf.predict(dt, to_dev(th0), thf, fef, fif)
    for k in range(n_iter):
        pf.iterate(dt, thf, fef, fif, last=(k == n_iter - 1))
    got = to_host(thf)[:, -1].reshape(n_ts, M, 3, -1)
    for mem in range(M):
        ref = opf.run(of, oc, sdc.SDC(nf), sdc.SDC(nc), dt, th0[mem], n_ts, n_iter)
        for n in range(n_ts):
            assert np.all(rel_err(got[n, mem], ref.end_values[-1][n]) <= 1e-11), (mem, n)


def test_graph_replay_and_level_swap_match_direct_launches():
    """Iterations replayed from captured graphs equal direct launches bit for
    bit, and swapping in levels of another precision keeps the state."""
    import torch
    Tf, Tc, nf, nc, dt, n_ts = 15, 7, 5, 3, 300.0, 4
    gf, gc, _, _ = _levels(Tf, Tc, nf, nc, n_ts, (24, 48), (12, 24))
    gf32 = pfsh.Level(Tf, 24, 48, nf, max_batch=n_ts, precision="fp32")
    th0 = to_dev(seeded(Tf, (70,)))
    outs = []
    stream = torch.cuda.Stream()
    for graphs in (False, True):
        pf = pfsh.Pfasst(gf, gc, n_ts)
        pf.set_graphs(graphs)
        thf, fef, fif = gf.space_time(n_ts), gf.space_time(n_ts), gf.space_time(n_ts)
        with torch.cuda.stream(stream):
            for rep in range(2):        # the second block replays the captured graphs
                pf.set_levels(gf32, gc)
                pf.predict(dt, th0, thf, fef, fif)
                for k in range(4):
                    if k == 2:
                        pf.set_levels(gf, gc)
                    pf.iterate(dt, thf, fef, fif, last=(k == 3))
            stream.synchronize()
        outs.append(to_host(thf))
        pf.close()
    assert np.array_equal(outs[0], outs[1])
    with pytest.raises(pfsh.PfshError):
        pf2 = pfsh.Pfasst(gf, gc, n_ts)
        pf2.set_levels(gc, gc)      # wrong geometry for the fine level


@pytest.mark.parametrize("n_ts,n_iter,members", [(4, 4, 1), (3, 5, 2), (1, 3, 1), (5, 2, 1)])
def test_wavefront_run_equals_iteration_order(n_ts, n_iter, members):
    """The wavefront schedule performs the arithmetic of Algorithm 1 in another
    order: results equal the iteration-by-iteration calls bit for bit."""
    import torch
    Tf, Tc, nf, nc, dt = 15, 7, 5, 3, 300.0
    B = n_ts * members
    gf, gc, _, _ = _levels(Tf, Tc, nf, nc, B, (24, 48), (12, 24))
    th0 = to_dev(seeded(Tf, tuple(range(80, 80 + members))))
    outs = []
    stream = torch.cuda.Stream()
    for mode in ("iterate", "run", "run_graph"):
        pf = pfsh.Pfasst(gf, gc, n_ts, members)
        pf.set_graphs(mode == "run_graph")
        thf, fef, fif = gf.space_time(B), gf.space_time(B), gf.space_time(B)
        with torch.cuda.stream(stream):
            for rep in range(2 if mode == "run_graph" else 1):
                pf.predict(dt, th0, thf, fef, fif)
                if mode == "iterate":
                    for k in range(n_iter):
                        pf.iterate(dt, thf, fef, fif, last=(k == n_iter - 1))
                else:
                    pf.run(dt, thf, fef, fif, n_iter)
            stream.synchronize()
        outs.append((to_host(thf), to_host(fef), to_host(fif)))
        pf.close()
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)


def test_wavefront_with_fp64_finish_tracks_fp64():
    Tf, Tc, nf, nc, dt, n_ts = 31, 15, 5, 3, 120.0, 6
    gf, gc, _, _ = _levels(Tf, Tc, nf, nc, n_ts, (48, 96), (24, 48))
    gf32 = pfsh.Level(Tf, 48, 96, nf, max_batch=n_ts, precision="fp32")
    th0 = to_dev(seeded(Tf, (90,)))
    res = []
    for fine, alt in ((gf, None), (gf32, gf)):
        pf = pfsh.Pfasst(fine, gc, n_ts)
        thf, fef, fif = gf.space_time(n_ts), gf.space_time(n_ts), gf.space_time(n_ts)
        pf.predict(dt, th0, thf, fef, fif)
        pf.run(dt, thf, fef, fif, 6, fine_alt=alt, k_switch=4)
        res.append(to_host(thf)[:, -1])
        pf.close()
    err = np.max([rel_err(res[1][n], res[0][n]) for n in range(n_ts)], axis=0)
    assert np.all(err <= 1e-6), err
