"""Theoretical cost of PFASST-SH, serial SDC and MLSDC-SH (Sec. 5.5).

Costs are counted in units of one fine operator application, under the paper's
simplifications: solving the implicit system, evaluating F_I and evaluating
F_E all cost 1 on the fine level (eq. unusual_assumption), and a coarse
operator costs alpha^2 of the fine one, alpha = R_c / R_f the ratio of zonal
wavenumber counts (eq. assumption_coarsening_ratio).  Communication is not
counted.  Names follow the paper: n_ts time steps per block, M_f + 1 and
M_c + 1 Lobatto nodes, N_PF PFASST iterations, N_S SDC sweeps, N_ML MLSDC
iterations.
"""


def coarse_cost_ratio(R_f, R_c):
    """K_c / K_f = R_c (R_c + 1) / (R_f (R_f + 1)), the exact form of
    eq. assumption_coarsening_ratio (about alpha^2)."""
    return R_c * (R_c + 1) / (R_f * (R_f + 1))


def pfasst_cost(n_ts, M_f, M_c, N_PF, alpha):
    """Per-processor cost of PFASST(n_ts, M_f+1, M_c+1, N_PF, alpha):
    prediction (eqs. cost_initialization_pfasst_*: coarse F at all nodes after
    the restriction, coarse F at node 0 for each received initial condition,
    n_ts serial coarse sweeps) plus N_PF iterations (eqs. cost_iteration_pfasst_*:
    fine sweep, coarse F at the nodes but the first after the restriction,
    coarse F at node 0 after the receive, coarse sweep, fine F at node 0 after
    the new initial condition), eq. total_computational_cost_parallel_pfasst."""
    c = alpha * alpha
    pred = (M_c + 1) * 2 * c + n_ts * 2 * c + n_ts * M_c * 3 * c
    it = M_f * 3 + M_c * 2 * c + 2 * c + M_c * 3 * c + 2
    return {"pred": pred, "iter": it, "total": pred + N_PF * it}


def sdc_cost(n_ts, M_f, N_S):
    """Serial SDC(M_f+1, N_S) over the same n_ts steps (eq.
    computational_cost_serial_sdc): F at the start of each step's nodes and
    N_S sweeps of M_f implicit solves and evaluations."""
    return n_ts * M_f * 2 + n_ts * N_S * M_f * 3


def mlsdc_cost(n_ts, M_f, M_c, N_ML, alpha):
    """Serial MLSDC(M_f+1, M_c+1, N_ML, alpha) over n_ts steps: the SDC cost
    with N_ML fine sweeps plus, per iteration, the coarse F at M_c nodes after
    the restriction and a coarse sweep, 5 M_c alpha^2 (the coarse term that
    eq. speedup_pfasst_mlsdc adds to eq. speedup_pfasst_sdc)."""
    return sdc_cost(n_ts, M_f, N_ML) + 5 * n_ts * N_ML * M_c * alpha * alpha


def _abcd(n_ts, M_f, M_c):
    den = 3 * n_ts * M_f
    return (2 / 3, (3 * M_f + 2) / den, (5 * M_c + 2) / den,
            (2 * M_c + (3 * M_c + 2) * n_ts + 2) / den)


def speedup_vs_sdc(n_ts, M_f, M_c, N_PF, alpha, N_S, dt_ratio=1.0):
    """S_S of eq. speedup_pfasst_sdc, (N_S + a) / (b N_PF + c alpha^2 N_PF + d alpha^2),
    rescaled by dt_ratio = dt_PF / dt_SDC when the two schemes reach the same
    accuracy with different time steps."""
    a, b, c, d = _abcd(n_ts, M_f, M_c)
    a2 = alpha * alpha
    return dt_ratio * (N_S + a) / (b * N_PF + c * a2 * N_PF + d * a2)


def speedup_vs_mlsdc(n_ts, M_f, M_c, N_PF, alpha, N_ML, dt_ratio=1.0):
    """S_ML of eq. speedup_pfasst_mlsdc (same alpha for both schemes), with
    e = (3 M_f + 2)/(5 n_ts M_c), f = (5 M_c + 2)/(5 n_ts M_c),
    g = (2 M_c + (3 M_c + 2) n_ts + 2)/(5 n_ts M_c)."""
    a, b, c, d = _abcd(n_ts, M_f, M_c)
    den = 5 * n_ts * M_c
    e, f, g = (3 * M_f + 2) / den, (5 * M_c + 2) / den, (2 * M_c + (3 * M_c + 2) * n_ts + 2) / den
    a2 = alpha * alpha
    return dt_ratio * ((N_ML + a) / (b * N_PF + c * a2 * N_PF + d * a2)
                       + N_ML / (e * N_PF / a2 + f * N_PF + g))
