"""Host-side validation on real levels: every call rejects empty and
oversized inputs and inconsistent level pairs with its status code before it
enqueues anything, and the level keeps working afterwards (results after a
rejected call equal those before it, bit for bit)."""

import ctypes

import numpy as np
import pytest
import torch

from paper_1904_05988_amd import pfsh
from tests._gpu import seeded, to_dev, to_host

pytestmark = pytest.mark.gpu

EINVAL, ESHAPE = -1, -2


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


@pytest.fixture(scope="module")
def levels():
    gf = pfsh.Level(31, 48, 96, 3, max_batch=4)
    gc = pfsh.Level(15, 24, 48, 2, max_batch=4)
    yield gf, gc
    gf.close()
    gc.close()


def test_empty_and_oversized_batches_are_rejected(levels):
    gf, _ = levels
    L, h = pfsh.lib(), gf.handle
    x = to_dev(seeded(31, range(4)))
    th, fe, fi = gf.space_time(4), gf.space_time(4), gf.space_time(4)
    grid = torch.empty((20, 48, 96), dtype=torch.float64, device="cuda")
    for b in (0, -1, 5):
        assert L.pfsh_rhs(h, _p(x), _p(fe), _p(fi), b, None) == ESHAPE
        assert L.pfsh_implicit_solve(h, 10.0, _p(x), _p(fe), b, None) == ESHAPE
        assert L.pfsh_sdc_sweep(h, 60.0, _p(th), _p(fe), _p(fi), None, b, None) == ESHAPE
        assert L.pfsh_spread(h, _p(th), _p(fe), _p(fi), b, None) == ESHAPE
    out = torch.empty((4, 3), dtype=torch.float64, device="cuda")
    assert L.pfsh_residual(h, 60.0, _p(th), _p(fe), _p(fi), None, _p(out), 0, None) == ESHAPE
    for nf in (0, 17):     # at most 4 * max_batch fields for the synthesis
        assert L.pfsh_sh_synthesis(h, _p(x), _p(grid), nf, None) == ESHAPE
    assert L.pfsh_sh_analysis(h, _p(grid), _p(x), 21, None) == ESHAPE   # 5 * max_batch


def test_bad_scalars_are_rejected(levels):
    gf, _ = levels
    L, h = pfsh.lib(), gf.handle
    th, fe, fi = gf.space_time(1), gf.space_time(1), gf.space_time(1)
    for dt in (0.0, -60.0, float("nan"), float("inf")):
        assert L.pfsh_sdc_sweep(h, dt, _p(th), _p(fe), _p(fi), None, 1, None) == EINVAL
    for beta in (-1.0, float("nan")):
        assert L.pfsh_implicit_solve(h, beta, _p(th), _p(fe), 1, None) == EINVAL
    assert L.pfsh_level_set_implicit(h, 2) == EINVAL
    assert L.pfsh_level_set_variant(h, 0, 1, 99) == EINVAL
    assert L.pfsh_level_set_variant(h, 0, 5, 0) == ESHAPE          # batch > max_batch


def test_inconsistent_level_pairs_are_rejected(levels):
    gf, gc = levels
    L = pfsh.lib()
    a = gf.space_time(4)
    c = gc.space_time(4)
    # the "coarse" level must not be finer than the fine one
    assert L.pfsh_restrict(gc.handle, gf.handle, _p(c), _p(a), 1, None) == ESHAPE
    assert L.pfsh_restrict(gf.handle, gc.handle, _p(a), _p(c), 5, None) == ESHAPE
    h = ctypes.c_void_p()
    assert L.pfsh_pfasst_create(gf.handle, gc.handle, 5, 1, ctypes.byref(h)) != 0   # 5 > max_batch
    assert not h.value


def test_level_still_works_after_rejected_calls(levels):
    gf, _ = levels
    x = to_dev(seeded(31, range(2)))
    fe0, fi0 = gf.rhs(x)
    ref = to_host(fe0), to_host(fi0)
    L, h = pfsh.lib(), gf.handle
    assert L.pfsh_rhs(h, _p(x), _p(fe0), _p(fi0), 9, None) == ESHAPE
    assert L.pfsh_sdc_sweep(h, -1.0, _p(x), _p(fe0), _p(fi0), None, 1, None) == EINVAL
    fe1, fi1 = gf.rhs(x)
    assert np.array_equal(to_host(fe1), ref[0]) and np.array_equal(to_host(fi1), ref[1])
