"""The kernel-timing diagnostic (pfsh_profile_enable / pfsh_profile_read):
every profiled launch is counted once, its time is the kernel's own (positive,
within the wall time of the calls), the batch filter splits the launches, and
profiling changes no result bit."""

import time

import numpy as np
import pytest
import torch

from paper_1904_05988_amd import pfsh
from tests._gpu import seeded, to_dev, to_host

pytestmark = pytest.mark.gpu

KERNELS = ("leg_synth", "ring", "leg_anal", "assemble", "prep", "sweep_node")


def _sweep(gl, th0, profile):
    B = th0.shape[0]
    th, fe, fi = gl.space_time(B), gl.space_time(B), gl.space_time(B)
    gl.profile(profile)
    e, i = gl.rhs(th0)
    th[:, 0], fe[:, 0], fi[:, 0] = th0, e, i
    gl.spread(th, fe, fi)
    gl.sdc_sweep(100.0, th, fe, fi)
    return to_host(th), to_host(fe)


@pytest.mark.parametrize("B", [2, 5])
def test_launch_counts_times_and_bits(B):
    """T31 on 48 x 96, 3 nodes.  Batch 2 takes the fused per-order node (one
    launch per node and a last one for F_E of node 2, a ring stage after each
    node); batch 5 the separate kernels (per node: sweep node, synthesis, ring,
    analysis; then the assembly of node 2)."""
    gl = pfsh.Level(31, 48, 96, 3, max_batch=B)
    th0 = to_dev(seeded(31, range(40, 40 + B)))
    ref = _sweep(gl, th0, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    got = _sweep(gl, th0, True)
    wall_ms = (time.perf_counter() - t0) * 1e3
    counts = {k: gl.profile_read(k) for k in KERNELS}
    by_batch = {k: gl.profile_read(k, batch=B)[0] for k in KERNELS}
    other = {k: gl.profile_read(k, batch=B + 1)[0] for k in KERNELS}
    gl.profile(False)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    fused = B <= 2
    want = {"prep": 1, "leg_synth": 1 + (0 if fused else 2), "ring": 1 + 2,
            "leg_anal": 1 + (0 if fused else 2), "assemble": 1 + (0 if fused else 1),
            "sweep_node": 3 if fused else 2}
    for k in KERNELS:
        n, ms = counts[k]
        assert n == want[k], (k, n, want[k])
        assert 0.0 < ms < wall_ms, (k, ms, wall_ms)
        # every launch here was over B states
        assert by_batch[k] == n and other[k] == 0, (k, by_batch[k], other[k])
