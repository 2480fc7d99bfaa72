"""Pins of the oracle's MLSDC-SH comparator (Sec. 5.5) and of the cost-model
helper (Sec. 5.5, eqs. total_computational_cost_parallel_pfasst,
computational_cost_serial_sdc, speedup_pfasst_sdc, speedup_pfasst_mlsdc).

MLSDC pins: converged, it reaches the serial SDC collocation solution of every
step; with the coarse level equal to the fine level (identity transfers, tau =
0 up to rounding) an iteration is two fine sweeps; a planted mistake (tau
dropped) moves its fixed point.  Cost-model pins: the closed-form speedups
equal the ratios of the term-by-term costs, and they agree within 25% with the
speedups the paper observed (Tables of Sec. 6; the paper reports them as
consistent with the model)."""

import numpy as np
import pytest

from oracle import mlsdc, sdc, swe, transfer
from paper_1904_05988_amd import costmodel, inputs

TF, TC = 10, 5


@pytest.fixture(scope="module")
def levels():
    return swe.Level(TF, 16, 32), swe.Level(TC, 8, 18)


def test_converged_mlsdc_is_serial_collocation(levels):
    lf, lc = levels
    sf, sc = sdc.SDC(5), sdc.SDC(3)
    th0 = inputs.seeded_state(TF, 31)
    ends = mlsdc.run(lf, lc, sf, sc, 300.0, th0, 2, 25)
    ref = sdc.serial_sdc(lf, sf, 300.0, th0, 2, 40)
    scale = np.abs(ref).max(axis=1)
    scale[0] = np.abs(ref[0, 1:]).max()
    assert np.all(np.abs(ends[-1] - ref).max(axis=1) <= 1e-12 * scale)


def test_identity_coarse_level_gives_two_sweeps_per_iteration(levels):
    lf, _ = levels
    sf = sdc.SDC(3)
    th0 = inputs.seeded_state(TF, 32)
    ends = mlsdc.run(lf, lf, sf, sdc.SDC(3), 200.0, th0, 1, 2)
    ref = sdc.serial_sdc(lf, sf, 200.0, th0, 1, 4)
    scale = np.abs(ref).max(axis=1)
    scale[0] = np.abs(ref[0, 1:]).max()
    assert np.all(np.abs(ends[-1] - ref).max(axis=1) <= 1e-13 * scale)


def test_planted_mistake_without_tau_is_caught(levels, monkeypatch):
    lf, lc = levels
    sf, sc = sdc.SDC(5), sdc.SDC(3)
    th0 = inputs.seeded_state(TF, 31)
    ref = sdc.serial_sdc(lf, sf, 300.0, th0, 1, 40)
    monkeypatch.setattr(transfer, "fas_tau", lambda *a: np.zeros_like(a[7]))
    ends = mlsdc.run(lf, lc, sf, sc, 300.0, th0, 1, 25)
    scale = np.abs(ref).max(axis=1)
    scale[0] = np.abs(ref[0, 1:]).max()
    assert np.any(np.abs(ends[-1] - ref).max(axis=1) > 1e-9 * scale)


# ----------------------------------------------------------------- cost model
@pytest.mark.parametrize("nts,mf,mc,npf,alpha,ns", [(16, 2, 1, 4, 0.2, 4), (16, 4, 2, 8, 0.8, 8),
                                                     (16, 4, 2, 16, 1.0, 8), (4, 4, 2, 3, 0.5, 6)])
def test_closed_form_speedups_equal_cost_ratios(nts, mf, mc, npf, alpha, ns):
    ratio = costmodel.sdc_cost(nts, mf, ns) / costmodel.pfasst_cost(nts, mf, mc, npf, alpha)["total"]
    assert costmodel.speedup_vs_sdc(nts, mf, mc, npf, alpha, ns) == pytest.approx(ratio, rel=1e-13)
    ratio_ml = (costmodel.mlsdc_cost(nts, mf, mc, ns, alpha)
                / costmodel.pfasst_cost(nts, mf, mc, npf, alpha)["total"])
    assert costmodel.speedup_vs_mlsdc(nts, mf, mc, npf, alpha, ns) == pytest.approx(ratio_ml, rel=1e-13)


# (PFASST (n_ts, M_f+1, M_c+1, N_PF, alpha), dt) vs (SDC (M_f+1, N_S), dt) and
# (MLSDC (M_f+1, M_c+1, N_ML, alpha), dt): the observed speedups S_S, S_ML the
# paper prints for the Gaussian dome, Rossby-Haurwitz and Galewsky runs
OBSERVED = [((16, 3, 2, 4, 1 / 5), 128, (3, 4), 400, 4.1, (3, 2, 2, 1 / 2), 400, 3.0),
            ((16, 5, 3, 8, 4 / 5), 100, (5, 8), 200, 3.7, (5, 3, 4, 1 / 2), 200, 2.5),
            ((16, 3, 2, 4, 1 / 5), 100, (3, 4), 400, 3.2, (3, 2, 2, 1 / 2), 400, 2.2),
            ((16, 5, 3, 8, 1 / 2), 320, (5, 8), 640, 5.2, (5, 3, 4, 1 / 2), 640, 3.6),
            ((16, 5, 3, 16, 1.0), 240, (5, 8), 240, 3.7, (5, 3, 4, 4 / 5), 60, 10.7)]


@pytest.mark.parametrize("row", OBSERVED)
def test_model_speedups_agree_with_observed(row):
    (nts, nf, nc, npf, a_pf), dt_pf, (snf, ns), dt_s, s_obs, (mnf, mnc, nml, a_ml), dt_ml, ml_obs = row
    pf = costmodel.pfasst_cost(nts, nf - 1, nc - 1, npf, a_pf)["total"]
    s = costmodel.sdc_cost(nts, snf - 1, ns) / pf * dt_pf / dt_s
    ml = costmodel.mlsdc_cost(nts, mnf - 1, mnc - 1, nml, a_ml) / pf * dt_pf / dt_ml
    assert abs(s / s_obs - 1) <= 0.25, (s, s_obs)
    assert abs(ml / ml_obs - 1) <= 0.25, (ml, ml_obs)
    if snf == nf:   # the closed form (same node count) with the time-step rescaling
        closed = costmodel.speedup_vs_sdc(nts, nf - 1, nc - 1, npf, a_pf, ns, dt_pf / dt_s)
        assert closed == pytest.approx(s, rel=1e-13)


def test_exact_coarsening_ratio_of_the_model():
    """eq. assumption_coarsening_ratio: C_c / C_f = R_c (R_c + 1) / (R_f (R_f + 1))
    = alpha^2 (R_f + 1/alpha) / (R_f + 1), close to alpha^2 for R_f >= 256."""
    r = costmodel.coarse_cost_ratio(256, 128)
    assert r == pytest.approx(128 * 129 / (256 * 257), rel=1e-15)
    assert r == pytest.approx(0.25 * (256 + 2) / 257, rel=1e-15)
    assert abs(r / 0.25 - 1) < 0.01
