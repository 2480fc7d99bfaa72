"""GPU parity of the transform stages and right-hand sides against the oracle.

Sizes span several MFMA tiles and ragged tails: T15 on 24x48 (12 northern rings,
padded to 32), T31 on 48x96 (the small workload), T63 on 96x192 with a batch
whose column count is not a multiple of the 64-column tile."""

import numpy as np
import pytest

from oracle import sht, swe
from tests._gpu import DEV, level_pair, rel_err, seeded, to_dev, to_host

pytestmark = pytest.mark.gpu

GRIDS = [(15, 24, 48), (31, 48, 96), (63, 96, 192)]


@pytest.mark.parametrize("T,nlat,nlon", GRIDS)
def test_sh_synthesis_matches_oracle(T, nlat, nlon):
    gl, ol = level_pair(T, nlat, nlon, 3, max_batch=2)
    rng = np.random.default_rng(T)
    nf = 5
    spec = rng.standard_normal((nf, gl.K)) + 1j * rng.standard_normal((nf, gl.K))
    spec[:, : T + 1] = spec[:, : T + 1].real
    grid = to_host(gl.sh_synthesis(to_dev(spec)))
    for f in range(nf):
        ref = sht.synthesis(ol.g, spec[f])
        assert np.abs(grid[f] - ref).max() <= 1e-13 * np.abs(ref).max(), f


# FP32 bound: unit roundoff u = 2^-24; the coefficients and tables are rounded
# once each, every product once, the Legendre sums (<= 17 terms per parity at
# T31, two accumulation chains) and the 7 FFT stages add at most one rounding
# per step, so ~30 u relative to the field's size covers the worst case
# (measured on gfx950: 1.3-1.8e-7, about 3 u).
FIELD_COUNT_TOL = {"fp64": 1e-13, "fp32": 2e-6}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nf", [1, 9, 12])
def test_sh_synthesis_field_counts(nf, prec):
    """Field counts that leave partial 16-column tiles and partial groups of
    four fields in the ring stage, up to the level's limit (4 x max_batch), in
    both Fourier-workspace order groups (4 FP64, 8 FP32 orders): every field
    against the oracle."""
    T, nlat, nlon = 31, 48, 96
    gl, ol = level_pair(T, nlat, nlon, 3, max_batch=3, precision=prec)
    rng = np.random.default_rng(200 + nf)
    spec = rng.standard_normal((nf, gl.K)) + 1j * rng.standard_normal((nf, gl.K))
    spec[:, : T + 1] = spec[:, : T + 1].real
    grid = to_host(gl.sh_synthesis(to_dev(spec)))
    for f in range(nf):
        ref = sht.synthesis(ol.g, spec[f])
        assert np.abs(grid[f] - ref).max() <= FIELD_COUNT_TOL[prec] * np.abs(ref).max(), f


@pytest.mark.parametrize("T,nlat,nlon", GRIDS)
def test_sh_analysis_matches_oracle_and_round_trips(T, nlat, nlon):
    gl, ol = level_pair(T, nlat, nlon, 3, max_batch=2)
    rng = np.random.default_rng(100 + T)
    nf = 7
    grid = rng.standard_normal((nf, nlat, nlon))
    spec = to_host(gl.sh_analysis(to_dev(grid)))
    for f in range(nf):
        ref = sht.analysis(ol.g, grid[f])
        assert np.abs(spec[f] - ref).max() <= 1e-13 * np.abs(ref).max(), f
    # band-limited round trip on the device alone
    s0 = rng.standard_normal((3, gl.K)) + 1j * rng.standard_normal((3, gl.K))
    s0[:, : T + 1] = s0[:, : T + 1].real
    back = to_host(gl.sh_analysis(gl.sh_synthesis(to_dev(s0))))
    assert np.abs(back - s0).max() <= 1e-13 * np.abs(s0).max()


def test_single_harmonics_exact():
    T, nlat, nlon = 31, 48, 96
    gl, _ = level_pair(T, nlat, nlon, 3, max_batch=4)
    cases = [(0, 0), (0, 31), (5, 17), (31, 31), (12, 13)]
    spec = np.zeros((len(cases), gl.K), dtype=np.complex128)
    for i, (m, n) in enumerate(cases):
        spec[i, sht.index(T, m, n)] = 1.0 if m == 0 else (0.6 - 0.8j)
    back = to_host(gl.sh_analysis(gl.sh_synthesis(to_dev(spec))))
    np.testing.assert_allclose(back, spec, atol=2e-14)


@pytest.mark.parametrize("T,nlat,nlon,B", [(15, 24, 48, 3), (31, 48, 96, 2), (63, 96, 192, 5)])
def test_rhs_matches_oracle(T, nlat, nlon, B):
    gl, ol = level_pair(T, nlat, nlon, 3, max_batch=B)
    states = seeded(T, range(10, 10 + B))
    fe, fi = gl.rhs(to_dev(states))
    fe, fi = to_host(fe), to_host(fi)
    for b in range(B):
        rfe, rfi = swe.rhs(ol, states[b])
        assert np.all(rel_err(fe[b], rfe) <= 1e-12), (b, rel_err(fe[b], rfe))
        assert np.all(rel_err(fi[b], rfi) <= 1e-14), (b, rel_err(fi[b], rfi))


def test_rhs_batch_invariance_bitwise():
    T, nlat, nlon = 31, 48, 96
    gl, _ = level_pair(T, nlat, nlon, 3, max_batch=6)
    states = seeded(T, range(6))
    fe_all, _ = gl.rhs(to_dev(states))
    fe_all = to_host(fe_all)
    for b in (0, 3, 5):
        fe1, _ = gl.rhs(to_dev(states[b:b + 1]))
        assert np.array_equal(to_host(fe1)[0], fe_all[b])


def test_solid_body_steady_state_on_device():
    T, nlat, nlon = 31, 48, 96
    gl, _ = level_pair(T, nlat, nlon, 3, max_batch=1, nu=0.0)
    from paper_1904_05988_amd import inputs
    st = (inputs.mean_geopotential(T) + inputs.solid_body(T, 20.0))[None]
    fe, fi = gl.rhs(to_dev(st))
    fe, fi = to_host(fe)[0], to_host(fi)[0]
    scale = np.abs(fe).max()
    assert np.abs(fe + fi).max() <= 1e-13 * scale
    assert np.abs(fe[:, 0]).max() <= 1e-25    # global means are not forced


@pytest.mark.parametrize("beta", [0.0, 40.0, 1234.5])
def test_implicit_solve_matches_oracle(beta):
    T, nlat, nlon = 63, 96, 192
    gl, ol = level_pair(T, nlat, nlon, 3, max_batch=3)
    rng = np.random.default_rng(4)
    b = rng.standard_normal((3, 3, gl.K)) + 1j * rng.standard_normal((3, 3, gl.K))
    x = to_host(gl.implicit_solve(beta, to_dev(b)))
    for i in range(3):
        ref = swe.implicit_solve(ol, beta, b[i])
        np.testing.assert_allclose(x[i], ref, rtol=1e-14, atol=1e-300)
