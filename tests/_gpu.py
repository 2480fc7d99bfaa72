"""Helpers of the GPU parity tests: device levels next to oracle levels, and
the normalized error used to compare them."""

import numpy as np
import torch

from oracle import sdc, swe
from paper_1904_05988_amd import inputs
from paper_1904_05988_amd import pfsh

DEV = torch.device("cuda", 0)


def level_pair(T, nlat, nlon, nn, max_batch=1, precision="fp64", **phys):
    gl = pfsh.Level(T, nlat, nlon, nn, max_batch=max_batch, precision=precision, **phys)
    ol = swe.Level(T, nlat, nlon, swe.Physics(**phys) if phys else None)
    return gl, ol


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def to_host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_err(got, ref, axis_var=-2):
    """max |got - ref| / max |ref| per variable (Phi, zeta, delta), Phi without
    its (0,0) mean slot in the denominator."""
    got = np.moveaxis(np.asarray(got), axis_var, 0)
    ref = np.moveaxis(np.asarray(ref), axis_var, 0)
    out = []
    for v in range(3):
        den_src = ref[v].copy()
        if v == 0:
            den_src[..., 0] = 0.0
        den = np.abs(den_src).max()
        out.append(np.abs(got[v] - ref[v]).max() / (den if den > 0 else 1.0))
    return np.array(out)


def oracle_spread_batch(ol, states, nn):
    th, fe, fi = [], [], []
    for s in states:
        a, b, c = sdc.spread(ol, s, nn)
        th.append(a); fe.append(b); fi.append(c)
    return np.array(th), np.array(fe), np.array(fi)


def seeded(T, seeds, power=2.0):
    return inputs.seeded_batch(T, seeds, power)
