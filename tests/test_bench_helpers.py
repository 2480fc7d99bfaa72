"""CPU checks of bench.py's host logic: the algorithmic work models behind the
roofline (structure: flops and bytes linear in the batch, tables in the
intercept), the choice of the bound, the counter table's source digest, and
the error norms (the mean-geopotential slot out of both maxima)."""

import importlib.util
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_legendre_flops_count_every_degree_to_T_plus_1(bench):
    # pairs (m, n), m = 0..T, n = m..T+1: (T + 1)(T + 4) / 2
    for T, nlat in ((7, 12), (30, 48), (255, 384)):
        deg = (T + 1) * (T + 4) // 2
        assert bench.legendre_flops(T, nlat, 10) == 2.0 * deg * (nlat // 2) * 10


@pytest.mark.parametrize("kernel", ["leg_synth", "leg_anal", "ring", "prep", "assemble",
                                    "sweep_node"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_work_models_are_affine_in_the_batch(bench, kernel, prec):
    """Per launch: data terms grow with the batch, tables do not.  The
    batch-1/2 fused node has its own (fused) model, so batches 3..5 here."""
    w = [bench.kernel_work(kernel, 127, 192, 384, 3, b, prec) for b in (3, 4, 5)]
    for key in ("flops", "bytes"):
        d1, d2 = w[1][key] - w[0][key], w[2][key] - w[1][key]
        assert d1 == pytest.approx(d2, rel=1e-12)
    if kernel in ("leg_synth", "leg_anal"):
        intercept = w[0]["bytes"] - 3 * (w[1]["bytes"] - w[0]["bytes"])
        assert intercept == pytest.approx(bench.table_bytes(127, 192, prec), rel=1e-12)
    fused = bench.kernel_work("sweep_node", 127, 192, 384, 3, 1, prec)
    assert fused["symbol"].startswith("k_node_fused")
    assert fused["bytes"] > 2 * bench.table_bytes(127, 192, prec)


def test_roofline_names_the_resource_with_the_longer_time(bench):
    peak_f, peak_b = bench.PEAKS["fp32"] * 1e12, bench.HBM_PEAK * 1e9
    mfma_heavy = {"flops": 2.0 * peak_f * 1e-6, "bytes": 0.5 * peak_b * 1e-6}
    r = bench.roofline_of(mfma_heavy, 4e-6, "fp32")
    assert r["bound"] == "mfma" and r["frac"] == pytest.approx(0.5)
    assert r["other_bound"]["bound"] == "hbm" and r["other_bound"]["frac"] == pytest.approx(0.125)
    hbm_heavy = {"flops": 0.5 * peak_f * 1e-6, "bytes": 2.0 * peak_b * 1e-6}
    r = bench.roofline_of(hbm_heavy, 4e-6, "fp32")
    assert r["bound"] == "hbm" and r["frac"] == pytest.approx(0.5)
    assert r["algorithmic_time_us"] == pytest.approx(2.0)


def test_traffic_is_reported_only_for_the_digest_it_was_taken_on(bench, tmp_path, monkeypatch):
    digest = bench.source_digest(bench.KERNEL_SOURCES["sweep_node"])
    table = tmp_path / "traffic.md"
    row = "| `coarse_mixed/sweep_node/b1` | `k` | 1000 | 234 | `{}` | 1 | 2 | 3 | 4 |\n"
    dom = {"level": "coarse_mixed", "kernel": "sweep_node", "batch": 1}
    monkeypatch.setattr(bench, "TRAFFIC_TABLE", str(table))
    table.write_text("| head |\n" + row.format(digest))
    assert bench.measured_traffic(dom)[0] == 1234.0
    table.write_text(row.format("0000000000000000"))
    value, why = bench.measured_traffic(dom)
    assert value is None and "another source" in why
    assert bench.measured_traffic({**dom, "batch": 2})[0] is None
    table.unlink()
    assert bench.measured_traffic(dom) == (None, "no counter table")


def test_rel_err_leaves_the_mean_geopotential_out_of_both_maxima(bench):
    rng = np.random.default_rng(0)
    ref = rng.standard_normal((1, 3, 40)) + 1j * rng.standard_normal((1, 3, 40))
    ref[:, 0, 0] = 1e6
    got = ref.copy()
    got[:, 0, 0] += 1.0                      # only the mean slot differs
    assert bench.rel_err(got, ref) == [0.0, 0.0, 0.0]
    got[:, 2, 7] += 1e-3
    e = bench.rel_err(got, ref)
    assert e[0] == 0.0 and e[1] == 0.0
    assert e[2] == pytest.approx(1e-3 / np.abs(ref[:, 2]).max())


def test_oracle_block_error_on_its_own_sample(bench, monkeypatch):
    d = np.load(bench.GOLDEN)
    slots, final = d["slots"], d["final"]
    K = 256 * 257 // 2
    full = np.zeros((16, 3, K), complex)
    full[:, :, slots] = final
    assert bench.oracle_golden_err(full) == [0.0, 0.0, 0.0]
    full[3, 0, 0] += 1.0                       # the mean slot (sampled first) is left out
    assert bench.oracle_golden_err(full) == [0.0, 0.0, 0.0]
    full[5, 1, slots[40]] += 1e-6
    e = bench.oracle_golden_err(full)
    assert e[0] == 0.0 and e[2] == 0.0
    assert e[1] == pytest.approx(1e-6 / np.abs(final[5, 1]).max())
    monkeypatch.setattr(bench, "WORKLOAD", "pfasst_t511_t255_32x4_ensemble")
    assert bench.oracle_golden_err(full) is None
