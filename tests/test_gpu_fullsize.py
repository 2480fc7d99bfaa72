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


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_mixed_precision_sweep_error(t255_states, prec):
    """Transform stages in FP32 / split-BF16x3: after two sweeps the state
    differs from the FP64 path by <= 1e-6 (normalized per variable)."""
    g64 = pfsh.Level(*T255, 5, max_batch=4)
    gmx = pfsh.Level(*T255, 5, max_batch=4, precision=prec)
    states = t255_states[:4]
    a = _spread(g64, states)
    b = _spread(gmx, states)
    for _ in range(2):
        g64.sdc_sweep(60.0, *a)
        gmx.sdc_sweep(60.0, *b)
    x64, xmx = to_host(a[0]), to_host(b[0])
    fe64, femx = to_host(a[1]), to_host(b[1])
    for s in range(4):
        e = rel_err(xmx[s, -1], x64[s, -1])
        assert np.all(e <= 1e-6), (prec, s, e)
        ef = rel_err(femx[s, -1], fe64[s, -1])
        bound = 1e-4 if prec == "fp32" else 1e-3
        assert np.all(ef <= bound), (prec, s, ef)


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
