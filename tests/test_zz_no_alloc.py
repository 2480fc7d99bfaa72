"""The allocation-free residual entry point (pfsh_residual_noalloc) through the
C ABI, against the existing entry point (pfsh_residual) on the same inputs.

The two launch the same kernels in the same order, so their outputs agree bit
for bit; the allocation-free call keeps its partial maxima in the library's
static device array, shared by every call on the GPU, so consecutive calls of
different sizes (the second smaller) are compared, as are the largest accepted
size and the first rejected one."""

import ctypes

import numpy as np
import pytest
import torch

from paper_1904_05988_amd import pfsh

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
SCRATCH = 1 << 19          # PFSH_RESIDUAL_SCRATCH_DOUBLES
ESHAPE = -2


def _arrays(B, nn, K, seed, scale=1.0):
    g = torch.Generator(device=DEV).manual_seed(seed)

    def one():
        return (torch.randn((B, nn, 3, K), dtype=torch.complex128, device=DEV, generator=g) * scale)
    return one(), one(), one(), one()


def _call(fn, gl, dt, th, fe, fi, tau, out):
    B = th.shape[0]
    s = ctypes.c_void_p(torch.cuda.current_stream(DEV).cuda_stream)
    return fn(gl.handle, ctypes.c_double(dt), ctypes.c_void_p(th.data_ptr()),
              ctypes.c_void_p(fe.data_ptr()), ctypes.c_void_p(fi.data_ptr()),
              None if tau is None else ctypes.c_void_p(tau.data_ptr()),
              ctypes.c_void_p(out.data_ptr()), B, s)


def _both(gl, dt, th, fe, fi, tau):
    lib = pfsh.lib()
    B = th.shape[0]
    ref = torch.full((B, 3), -1.0, dtype=torch.float64, device=DEV)
    got = torch.full((B, 3), -2.0, dtype=torch.float64, device=DEV)
    assert _call(lib.pfsh_residual, gl, dt, th, fe, fi, tau, ref) == 0
    assert _call(lib.pfsh_residual_noalloc, gl, dt, th, fe, fi, tau, got) == 0
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_residual_equals_residual_on_consecutive_calls():
    big = pfsh.Level(63, 96, 192, 5, max_batch=6)
    small = pfsh.Level(15, 24, 48, 3, max_batch=2)
    calls = [(big, 6, 60.0, True, 1), (small, 2, 300.0, False, 2), (big, 1, 60.0, False, 3),
             (small, 1, 120.0, True, 4)]
    for gl, B, dt, with_tau, seed in calls:
        th, fe, fi, tau = _arrays(B, gl.n_nodes, gl.K, seed, 1e-3)
        ref, got = _both(gl, dt, th, fe, fi, tau if with_tau else None)
        assert np.all(np.isfinite(ref)) and np.all(ref > 0)
        np.testing.assert_array_equal(got, ref)
    # a NaN in one slice reaches that slice's entry only, in both entry points
    gl = big
    th, fe, fi, tau = _arrays(4, gl.n_nodes, gl.K, 9, 1e-3)
    fe[2, 3, 1, 17] = complex(float("nan"), 0.0)
    ref, got = _both(gl, 60.0, th, fe, fi, None)
    assert np.isnan(got[2, 1]) and np.isnan(ref[2, 1])
    np.testing.assert_array_equal(np.isnan(got), np.isnan(ref))
    np.testing.assert_array_equal(got[~np.isnan(got)], ref[~np.isnan(ref)])


def test_noalloc_residual_largest_size_and_rejection():
    """T31, 2 nodes: the partial maxima take 3 ceil(528 / 256) = 9 doubles per
    slice, so 58254 slices fill the static scratch and 58255 are rejected
    before anything runs.  The largest call is checked against the existing
    entry point run in chunks of at most 4096 slices (slices are independent),
    then a smaller call follows."""
    gl = pfsh.Level(31, 48, 96, 2, max_batch=4096)
    per = 3 * ((gl.K + 255) // 256)
    limit = SCRATCH // per
    assert limit == 58254
    lib = pfsh.lib()
    th, fe, fi, _ = _arrays(limit + 1, 2, gl.K, 11, 1e-3)
    out = torch.zeros((limit + 1, 3), dtype=torch.float64, device=DEV)
    assert _call(lib.pfsh_residual_noalloc, gl, 60.0, th, fe, fi, None, out) == ESHAPE
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0          # nothing was enqueued
    a, b, c = th[:limit], fe[:limit], fi[:limit]
    got = torch.zeros((limit, 3), dtype=torch.float64, device=DEV)
    assert _call(lib.pfsh_residual_noalloc, gl, 60.0, a, b, c, None, got) == 0
    ref = torch.zeros_like(got)
    for s in range(0, limit, 4096):
        e = min(limit, s + 4096)
        assert _call(lib.pfsh_residual, gl, 60.0, a[s:e], b[s:e], c[s:e], None, ref[s:e]) == 0
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got.cpu().numpy(), ref.cpu().numpy())
    del th, fe, fi, a, b, c
    th, fe, fi, _ = _arrays(3, 2, gl.K, 12, 1e-3)
    r1, g1 = _both(gl, 60.0, th, fe, fi, None)
    np.testing.assert_array_equal(g1, r1)
