"""Full-size GPU checks: the T255 x 16-slice sweep in the launch configuration
the benchmark times (sampled slices against the oracle, invariants on all),
the mixed-precision paths against FP64, and the zonal-jet serial SDC run
against its stored oracle reference."""

import os

import numpy as np
import pytest

from oracle import sdc, swe
from paper_1904_05988_amd import inputs, pfsh
from tests._gpu import rel_err, to_dev, to_host
from tests._ics import jet_state

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
T255 = (255, 384, 768)


def _spread(gl, states):
    B = states.shape[0]
    th, fe, fi = gl.space_time(B), gl.space_time(B), gl.space_time(B)
    th[:, 0] = to_dev(states)
    e, i = gl.rhs(to_dev(states))
    fe[:, 0] = e
    fi[:, 0] = i
    gl.spread(th, fe, fi)
    return th, fe, fi


@pytest.fixture(scope="module")
def t255_states():
    return inputs.seeded_batch(255, range(300, 316))


def test_t255_b16_sweep_sampled_against_oracle(t255_states):
    gl = pfsh.Level(*T255, 5, max_batch=16)
    th, fe, fi = _spread(gl, t255_states)
    gl.sdc_sweep(60.0, th, fe, fi)
    gth, gfe = to_host(th), to_host(fe)
    ol = swe.Level(*T255)
    sd = sdc.SDC(5)
    for b in (0, 15):
        rth, rfe, rfi = sdc.spread(ol, t255_states[b], 5)
        rth, rfe, rfi = sdc.sweep(ol, sd, 60.0, rth, rfe, rfi)
        for i in range(5):
            assert np.all(rel_err(gth[b, i], rth[i]) <= 1e-12), (b, i)
            assert np.all(rel_err(gfe[b, i], rfe[i]) <= 1e-11), (b, i)
    # invariant on every slice: the mean geopotential does not move
    for b in range(16):
        assert np.abs(gth[b, :, 0, 0] - gth[b, 0, 0, 0]).max() <= 1e-15 * abs(gth[b, 0, 0, 0])


# bounds per variable (Phi, zeta, delta) after two sweeps from the spread guess,
# each normalized by that slice's own maximum.  The divergence shows transform
# rounding most: its high-degree tendencies carry the kinetic-energy Laplacian
# (factor n(n+1)/a^2) and the gravity-wave response to geopotential errors,
# while its own amplitude is small (down to 3e-7 1/s in seed 303).
# FP32: the measured errors on gfx950 (7e-9, 4.5e-8, 1.9e-5) with a margin of
# 2-4.  BF16x3 from the arithmetic: its operands keep 16 significant bits
# (hi + lo, the lo*lo product dropped) where FP32 keeps 24, so its rounding per
# product is 2^8 = 256 times FP32's, and the FP32 errors scaled by 256 give
# (1.8e-6, 1.2e-5, 4.9e-3), rounded up; measured (3.7e-7, 1.5e-6, 1.0-1.1e-3).
SWEEP_BOUNDS = {"fp32": (2e-8, 2e-7, 5e-5), "bf16x3": (2e-6, 1.2e-5, 5e-3)}


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_mixed_precision_sweep_error(t255_states, prec):
    """Transform stages in FP32 / split-BF16x3 against the FP64 path after two
    sweeps, and a third sweep in FP64 that pulls the mixed iterate back."""
    g64 = pfsh.Level(*T255, 5, max_batch=4)
    gmx = pfsh.Level(*T255, 5, max_batch=4, precision=prec)
    states = t255_states[:4]
    a = _spread(g64, states)
    b = _spread(gmx, states)
    for _ in range(2):
        g64.sdc_sweep(60.0, *a)
        gmx.sdc_sweep(60.0, *b)
    x64, xmx = to_host(a[0]), to_host(b[0])
    worst = np.zeros(3)
    for s in range(4):
        worst = np.maximum(worst, rel_err(xmx[s, -1], x64[s, -1]))
    assert np.all(worst <= np.array(SWEEP_BOUNDS[prec])), (prec, worst)
    # one FP64 sweep on the mixed iterate (node-0 F re-evaluated in FP64)
    th, fe, fi = (t.clone() for t in b)
    e, i = g64.rhs(th[:, 0].contiguous())
    fe[:, 0] = e
    fi[:, 0] = i
    g64.sdc_sweep(60.0, th, fe, fi)
    g64.sdc_sweep(60.0, *a)
    after = np.zeros(3)
    for s in range(4):
        after = np.maximum(after, rel_err(to_host(th)[s, -1], to_host(a[0])[s, -1]))
    assert np.all(after < worst), (prec, worst, after)


@pytest.mark.parametrize("n64,coarse_mixed,finish_coarse_fp64",
                         [(2, True, False), (2, True, True), (4, True, True), (2, False, True)])
def test_pfasst_mixed_block_with_fp64_finish_within_1e6(n64, coarse_mixed, finish_coarse_fp64):
    """PFASST(16, 5, 3, 8) at T255/T127 from seed 3: FP32 transforms on the
    fine level (and, with coarse_mixed, on the coarse level) for the first
    iterations, an FP64 fine level for the last n64, with the coarse level
    FP64 there too (finish_coarse_fp64) or still mixed (the benchmark's recipe:
    n64 = 2, FP32 coarse transforms throughout); the block ends within 1e-6 of
    the FP64 block (per variable), closer than all-FP32.  The modes the coarse
    level also carries (n <= 127) are pulled back to the FP64 iterate by the
    FP64 iterations; the rounding left above the coarse truncation is only
    carried along by the fine sweeps and the initial-condition chain, which is
    where the rest of the difference sits."""
    fine, coarse = (255, 384, 768, 5), (127, 192, 384, 3)
    th0 = to_dev(inputs.seeded_state(255, 3)[None])

    def block(prec, n64, cmix, cfin64):
        gfm = pfsh.Level(*fine, max_batch=16, precision=prec)
        gc64 = pfsh.Level(*coarse, max_batch=16)
        gcm = pfsh.Level(*coarse, max_batch=16, precision=prec) if cmix else gc64
        gf64 = pfsh.Level(*fine, max_batch=16)
        pf = pfsh.Pfasst(gfm, gcm, 16)
        th, fe, fi = gfm.space_time(16), gfm.space_time(16), gfm.space_time(16)
        pf.predict(60.0, th0, th, fe, fi)
        for k in range(8):
            if k == 8 - n64:
                pf.set_levels(gf64, gc64 if cfin64 else gcm)
            pf.iterate(60.0, th, fe, fi, last=(k == 7))
        pf.close()
        return to_host(th)[:, -1]

    ref = block("fp64", 0, False, True)
    got = block("fp32", n64, coarse_mixed, finish_coarse_fp64)
    pure = block("fp32", 0, coarse_mixed, True)
    n = np.concatenate([np.arange(m, 256) for m in range(256)])
    err, err_low, err_pure = np.zeros(3), np.zeros(3), np.zeros(3)
    for s in range(16):
        err = np.maximum(err, rel_err(got[s], ref[s]))
        err_pure = np.maximum(err_pure, rel_err(pure[s], ref[s]))
        # the same norm with the difference taken over n <= 127 only
        diff = got[s].copy()
        diff[:, n > 127] = ref[s][:, n > 127]
        err_low = np.maximum(err_low, rel_err(diff, ref[s]))
    print("n64", n64, "coarse mixed", coarse_mixed, "coarse FP64 in the finish", finish_coarse_fp64,
          "err", err, "low modes", err_low, "all FP32", err_pure)
    assert np.all(err <= 1e-6), err
    # low modes: each FP64 iteration pulls them further back (measured, seed 3:
    # divergence 1.6e-7 (FP64 coarse throughout) and 1.8e-7 (FP32 coarse in the
    # mixed iterations) after two FP64 iterations, 5e-9 after four).  With the
    # coarse level left in FP32 for the FP64 iterations (the benchmark's
    # recipe) the last coarse correction carries FP32 transform rounding into
    # them: 2.7e-7 measured, bounded by 4e-7; the total error is unchanged
    # (7.7e-7), the high modes dominate it.
    low_bound = 1e-7 if n64 >= 4 else (3e-7 if finish_coarse_fp64 else 4e-7)
    assert np.all(err_low <= low_bound), err_low
    assert np.all(err_low <= err), (err_low, err)
    assert err[2] < err_pure[2], (err, err_pure)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_mixed_precision_sht_round_trip(prec):
    T, nlat, nlon = 127, 192, 384
    gl = pfsh.Level(T, nlat, nlon, 3, max_batch=2, precision=prec)
    rng = np.random.default_rng(1)
    s0 = rng.standard_normal((4, gl.K)) + 1j * rng.standard_normal((4, gl.K))
    s0[:, : T + 1] = s0[:, : T + 1].real
    back = to_host(gl.sh_analysis(gl.sh_synthesis(to_dev(s0))))
    tol = 2e-5 if prec == "fp32" else 2e-4
    assert np.abs(back - s0).max() <= tol * np.abs(s0).max()


def test_jet_serial_sdc_against_stored_oracle():
    path = os.path.join(HERE, "golden", "jet_t127_sdc5x8_20x60s.npz")
    ref = np.load(path)
    T, nlat, nlon, nn, nsweep, nstep = (int(v) for v in ref["meta"][:6])
    dt = float(ref["meta"][6])
    seed = int(ref["meta"][7])
    gl = pfsh.Level(T, nlat, nlon, nn, max_batch=1)
    x = jet_state(T, nlat, nlon, seed)[None]
    for step in range(nstep):
        th, fe, fi = _spread(gl, x)
        for _ in range(nsweep):
            gl.sdc_sweep(dt, th, fe, fi)
        x = to_host(th)[:, -1].copy()
        if step == 0:
            assert np.all(rel_err(x[0], ref["first"]) <= 1e-12)
    assert np.all(rel_err(x[0], ref["final"]) <= 1e-11), rel_err(x[0], ref["final"])
