"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/pfsh.h declares, and validates arguments on the host before any HIP
call (no compute call is made here)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pfsh.h")
LIB = os.path.join(ROOT, "paper_1904_05988_amd", "libpfsh.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pfsh_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        pytest.fail("libpfsh.so is not built (python -m paper_1904_05988_amd.build)")
    from paper_1904_05988_amd import pfsh
    return pfsh.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n


def test_binding_signatures_cover_header():
    from paper_1904_05988_amd import pfsh
    assert set(declared_functions()) == set(pfsh._SIGS)


def _desc(**kw):
    from paper_1904_05988_amd.pfsh import LevelDesc
    base = dict(T=31, nlat=48, nlon=96, n_nodes=3, max_batch=4, radius=6.371e6, omega=7.292e-5,
                phibar=9.81e4, nu=1e5, precision=0)
    base.update(kw)
    return LevelDesc(**base)


@pytest.mark.parametrize("kw,code", [
    ({}, 0),
    ({"T": 255, "nlat": 384, "nlon": 768, "n_nodes": 5, "max_batch": 16}, 0),
    ({"T": 511, "nlat": 768, "nlon": 1536, "precision": 2}, 0),
    ({"nlat": 47}, -2),            # odd
    ({"nlat": 32}, -2),            # < T+2
    ({"nlon": 60}, -2),            # < 2T+2
    ({"nlon": 80}, -5),            # not 2^a or 3*2^a
    ({"nlon": 3072, "T": 700, "nlat": 1000}, -5),
    ({"n_nodes": 1}, -2),
    ({"n_nodes": 10}, -2),
    ({"max_batch": 0}, -2),
    ({"radius": -1.0}, -1),
    ({"nu": -1.0}, -1),
    ({"precision": 3}, -1),
    ({"T": 0}, -2),
    ({"precision": 0x100}, 0),      # FP64 with the Legendre recurrence
    ({"precision": 0x101}, 0),      # FP32 with the Legendre recurrence
    ({"precision": 0x102}, -1),     # BF16x3 has no recurrence mode
    ({"precision": 0x200}, -1),     # unknown flag
])
def test_desc_validation(L, kw, code):
    d = _desc(**kw)
    assert L.pfsh_level_desc_check(ctypes.byref(d)) == code


def test_null_arguments_rejected_without_gpu(L):
    P = ctypes.c_void_p
    one = P(16)
    assert L.pfsh_level_desc_check(None) == -1
    assert L.pfsh_level_create(None, 0, None) == -1
    assert L.pfsh_rhs(None, one, one, one, 1, None) == -1
    assert L.pfsh_sdc_sweep(None, 1.0, one, one, one, None, 1, None) == -1
    assert L.pfsh_implicit_solve(None, 1.0, one, one, 1, None) == -1
    assert L.pfsh_sh_synthesis(None, one, one, 1, None) == -1
    assert L.pfsh_sh_analysis(None, one, one, 1, None) == -1
    assert L.pfsh_residual(None, 1.0, one, one, one, None, one, 1, None) == -1
    assert L.pfsh_residual_noalloc(None, 1.0, one, one, one, None, one, 1, None) == -1
    assert L.pfsh_level_set_implicit(None, 0) == -1
    assert L.pfsh_level_bytes(None, None, None) == -1
    assert L.pfsh_restrict(None, None, one, one, 1, None) == -1
    assert L.pfsh_interpolate_add(None, None, one, None, one, 1, None) == -1
    assert L.pfsh_fas_tau(None, None, 1.0, one, one, one, one, one, 1, None) == -1
    assert L.pfsh_spread(None, one, None, None, 1, None) == -1
    assert L.pfsh_pfasst_create(None, None, 1, 1, None) == -1
    assert L.pfsh_pfasst_predict(None, 1.0, one, one, one, one, None) == -1
    assert L.pfsh_pfasst_iterate(None, 1.0, one, one, one, 0, None) == -1
    assert L.pfsh_check_finite(None, 3, None) == -1
    assert L.pfsh_check_finite(one, 0, None) == 0
    v = ctypes.c_int()
    assert L.pfsh_variant_count(None, 0) == -1
    assert L.pfsh_level_set_variant(None, 0, 1, 0) == -1
    assert L.pfsh_level_get_variant(None, 0, 1, ctypes.byref(v)) == -1
    assert L.pfsh_level_autotune(None, 1, 5, None, None) == -1
    assert L.pfsh_level_autotune_ex(None, 1, 5, 1, None, None) == -1
    L.pfsh_level_destroy(None)
    L.pfsh_pfasst_destroy(None)


def test_status_strings(L):
    for code in (0, -1, -2, -3, -4, -5, -6, 99):
        s = L.pfsh_status_string(code)
        assert isinstance(s, bytes) and len(s) > 0


def test_create_without_device_fails_cleanly(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    d = _desc()
    h = ctypes.c_void_p(1)
    code = L.pfsh_level_create(ctypes.byref(d), 0, ctypes.byref(h))
    assert code in (-1, -4) and not h.value
