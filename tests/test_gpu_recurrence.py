"""Recurrence mode (PFSH_LEGENDRE_RECURRENCE): Legendre contractions that
evaluate P_n^m inside the kernel by the two-degree recurrence instead of
reading stored tables (Sec. 3), against the oracle and against the
tabulated mode.

Small sizes against the oracle: T15 on 24x48, T30 on 48x96 (even T), T31 on
48x96 and T63 on 96x192 (several 64-degree slabs of order 0 in the synthesis,
ragged last chunks, batches whose column count is not a multiple of the
column tile); a PFASST block at T15/T7.  Full sizes against the tabulated
level on the same inputs: T255 on 384x768 with 16 slices and T511 on
768x1536 with 2 slices (two ring slabs of the FP32 analysis, three of FP64).

Tolerances: the float64 recurrence restarts every 32 degrees of one parity
and its error grows along the chunk to ~1e-13 of a ring's largest P value
(tests/test_recurrence_math.py), against ~1e-16 for the rounded 80-bit
tables, so the FP64 transforms and right-hand sides are held to 1e-12 (the
tabulated mode: 1e-13 / 1e-12); at full size the F_E tendencies, whose
derivative terms weight the high degrees, are held to the 1e-11 that the
tabulated FP64 level meets against the oracle at T255 and T511 (measured
recurrence against tables at T255: 0.9, 1.1 and 2.3e-12).  FP32 operands round P to 6e-8 either way;
the FP32 recurrence level is compared with the FP32 tabulated level, whose
operands differ only where the recurrence's 1e-13 error crosses a rounding
boundary, at 1e-6 of each variable's scale (the FP32 transform round-off)."""

import numpy as np
import pytest
import torch

from oracle import pfasst as opf
from oracle import sdc, sht, swe
from paper_1904_05988_amd import inputs, pfsh
from tests._gpu import rel_err, seeded, to_dev, to_host

pytestmark = pytest.mark.gpu

GRIDS = [(15, 24, 48), (30, 48, 96), (31, 48, 96), (63, 96, 192)]


def _rec(T, nlat, nlon, nn=3, B=2, precision="fp64"):
    return pfsh.Level(T, nlat, nlon, nn, max_batch=B, precision=precision, legendre="recurrence")


@pytest.mark.parametrize("variant", [0, 1, 2])
@pytest.mark.parametrize("T,nlat,nlon", GRIDS)
def test_sh_synthesis_and_analysis_match_oracle(T, nlat, nlon, variant):
    """Variant 0: the generate-once kernels (synthesis with 32 rings per
    workgroup, analysis with 8 waves); 1: one recurrence per column tile; 2:
    generate-once with 16 rings (synthesis) and 4 waves (analysis)."""
    gl = _rec(T, nlat, nlon)
    for b in (1, 2):
        gl.set_variant("synth", b, variant)
        gl.set_variant("anal", b, variant)
    g = sht.Grid(T, nlat, nlon)
    rng = np.random.default_rng(7 + T)
    nf = 5
    spec = rng.standard_normal((nf, gl.K)) + 1j * rng.standard_normal((nf, gl.K))
    spec[:, : T + 1] = spec[:, : T + 1].real
    grid = to_host(gl.sh_synthesis(to_dev(spec)))
    for f in range(nf):
        ref = sht.synthesis(g, spec[f])
        assert np.abs(grid[f] - ref).max() <= 1e-12 * np.abs(ref).max(), ("synthesis", f)
    fields = rng.standard_normal((7, nlat, nlon))
    back = to_host(gl.sh_analysis(to_dev(fields)))
    for f in range(7):
        ref = sht.analysis(g, fields[f])
        assert np.abs(back[f] - ref).max() <= 1e-12 * np.abs(ref).max(), ("analysis", f)


@pytest.mark.parametrize("variant", [0, 1, 2])
@pytest.mark.parametrize("T,nlat,nlon,B", [(15, 24, 48, 3), (30, 48, 96, 2), (63, 96, 192, 5),
                                           (31, 48, 96, 13)])
def test_rhs_matches_oracle(T, nlat, nlon, B, variant):
    """B = 13: 9 analysis and 7 synthesis column blocks, so every wave of the
    generate-once kernels runs more than one (ragged) column round."""
    gl = _rec(T, nlat, nlon, B=B)
    gl.set_variant("synth", B, variant)
    gl.set_variant("anal", B, variant)
    ol = swe.Level(T, nlat, nlon)
    states = seeded(T, range(20, 20 + B))
    fe, fi = gl.rhs(to_dev(states))
    fe, fi = to_host(fe), to_host(fi)
    for b in range(B):
        rfe, rfi = swe.rhs(ol, states[b])
        assert np.all(rel_err(fe[b], rfe) <= 1e-12), (b, rel_err(fe[b], rfe))
        assert np.all(rel_err(fi[b], rfi) <= 1e-14), b


@pytest.mark.parametrize("B", [1, 3])
def test_sweep_matches_oracle(B):
    """Two sweeps of 3 nodes at T31 (batch 1 takes the separate kernels: the
    fused per-order node needs the tables)."""
    T, nlat, nlon, nn, dt = 31, 48, 96, 3, 200.0
    gl = _rec(T, nlat, nlon, nn, B=B)
    ol = swe.Level(T, nlat, nlon)
    sd = sdc.SDC(nn)
    th0 = seeded(T, range(30, 30 + B))
    th, fe, fi = gl.space_time(B), gl.space_time(B), gl.space_time(B)
    e, i = gl.rhs(to_dev(th0))
    th[:, 0], fe[:, 0], fi[:, 0] = to_dev(th0), e, i
    gl.spread(th, fe, fi)
    for _ in range(2):
        gl.sdc_sweep(dt, th, fe, fi)
    got = to_host(th)
    for b in range(B):
        t, f, g = sdc.spread(ol, th0[b], nn)
        for _ in range(2):
            t, f, g = sdc.sweep(ol, sd, dt, t, f, g)
        for n in range(1, nn):
            assert np.all(rel_err(got[b, n], t[n]) <= 1e-11), (b, n, rel_err(got[b, n], t[n]))


def test_pfasst_block_matches_oracle():
    Tf, Tc, nf, nc, dt, n_ts, n_iter = 15, 7, 5, 3, 300.0, 4, 3
    gf = _rec(Tf, 24, 48, nf, B=n_ts)
    gc = _rec(Tc, 12, 24, nc, B=n_ts)
    of, oc = swe.Level(Tf, 24, 48), swe.Level(Tc, 12, 24)
    th0 = seeded(Tf, (51,))[0]
    ref = opf.run(of, oc, sdc.SDC(nf), sdc.SDC(nc), dt, th0, n_ts, n_iter)
    pf = pfsh.Pfasst(gf, gc, n_ts)
    thf, fef, fif = gf.space_time(n_ts), gf.space_time(n_ts), gf.space_time(n_ts)
    pf.predict(dt, to_dev(th0[None]), thf, fef, fif)
    for k in range(n_iter):
        pf.iterate(dt, thf, fef, fif, last=(k == n_iter - 1))
    got = to_host(thf)
    for n in range(n_ts):
        e = rel_err(got[n, -1], ref.end_values[n_iter - 1][n])
        assert np.all(e <= 1e-11), (n, e)
    pf.close()


def _fullsize(T, nlat, nlon, B, precision):
    tab = pfsh.Level(T, nlat, nlon, 5, max_batch=B, precision=precision)
    rec = pfsh.Level(T, nlat, nlon, 5, max_batch=B, precision=precision, legendre="recurrence")
    x = to_dev(inputs.seeded_batch(T, tuple(range(B))))
    fe_t, _ = tab.rhs(x)
    fe_r, _ = rec.rhs(x)
    fe_t, fe_r = to_host(fe_t), to_host(fe_r)
    err = np.max([rel_err(fe_r[b], fe_t[b]) for b in range(B)], axis=0)
    sizes = tab.bytes()[0], rec.bytes()[0]
    tab.close()
    rec.close()
    torch.cuda.empty_cache()
    return err, sizes


@pytest.mark.parametrize("precision,bound", [("fp64", 1e-11), ("fp32", 1e-6)])
def test_t255_rhs_matches_tabulated_level(precision, bound):
    err, (tb, rb) = _fullsize(255, 384, 768, 16, precision)
    print(precision, "T255 x 16 recurrence vs tables", err, "table bytes", tb, "recurrence bytes", rb)
    assert np.all(err <= bound), err
    assert rb * 4 < tb


@pytest.mark.parametrize("precision,bound", [("fp64", 1e-11), ("fp32", 1e-6)])
def test_t511_rhs_matches_tabulated_level(precision, bound):
    err, (tb, rb) = _fullsize(511, 768, 1536, 2, precision)
    print(precision, "T511 x 2 recurrence vs tables", err, "table bytes", tb, "recurrence bytes", rb)
    assert np.all(err <= bound), err
    assert rb * 4 < tb
