"""Two-level multi-level SDC, MLSDC-SH, over serial time steps (oracle; test
infrastructure).

Sec. 5.5 compares PFASST-SH with the serial SDC and MLSDC-SH schemes; the
MLSDC-SH iteration is described in the authors' earlier work and, per the
table of scheme parameters, involves one sweep on the fine level and one
sweep on the coarse level.  Reading taken here: every time step starts from
the spread initial guess on the fine level (node 0 = the step's initial
condition, F there evaluated) and runs N_ML iterations of
  A) a fine sweep;
  B) restriction to all coarse nodes (Sec. 5.3), coarse F at all nodes,
     copies of the restricted values, and the FAS correction tau_c (Sec. 5.1.2);
  C) a coarse FAS sweep from the restricted (fixed) initial condition;
  D) the interpolated coarse increments of Theta, F_E and F_I added at all
     fine nodes;
that is, one iteration of Algorithm 1 on a single time step with nothing to
send or receive.  The next step starts from the fine last-node value.  This
matches the work the cost model of Sec. 5.5 assigns to an MLSDC-SH iteration:
one fine sweep, coarse right-hand sides at the coarse nodes and one coarse
sweep, with no fine evaluation after the interpolation.
"""

import numpy as np

from . import sdc, swe, transfer


def _eval_all(lv, th, lin):
    fe = np.empty_like(th)
    fi = np.empty_like(th)
    for i in range(th.shape[0]):
        fe[i], fi[i] = swe.rhs(lv, th[i], lin)
    return fe, fi


def iteration(lv_f, lv_c, sd_f, sd_c, dt, th_f, fe_f, fi_f, linear_coriolis=False):
    """One MLSDC iteration (steps A-D above) on fine arrays [Mf+1, 3, Kf]."""
    Tf, Tc = lv_f.T, lv_c.T
    lin = linear_coriolis
    th_f, fe_f, fi_f = sdc.sweep(lv_f, sd_f, dt, th_f, fe_f, fi_f, None, lin)
    th_c = transfer.restrict(sd_f, sd_c, Tf, Tc, th_f)
    fe_c, fi_c = _eval_all(lv_c, th_c, lin)
    old = (th_c.copy(), fe_c.copy(), fi_c.copy())
    tau = transfer.fas_tau(sd_f, sd_c, Tf, Tc, dt, fe_f, fi_f, fe_c, fi_c)
    th_c, fe_c, fi_c = sdc.sweep(lv_c, sd_c, dt, th_c, fe_c, fi_c, tau, lin)
    th_f = th_f + transfer.interpolate(sd_c, sd_f, Tc, Tf, th_c - old[0])
    fe_f = fe_f + transfer.interpolate(sd_c, sd_f, Tc, Tf, fe_c - old[1])
    fi_f = fi_f + transfer.interpolate(sd_c, sd_f, Tc, Tf, fi_c - old[2])
    return th_f, fe_f, fi_f


def run(lv_f, lv_c, sd_f, sd_c, dt, theta0, nsteps, n_iter, linear_coriolis=False):
    """MLSDC(Mf+1, Mc+1, N_ML = n_iter, alpha) over nsteps steps of dt from
    theta0 [3, Kf]; returns the end value of every step [nsteps, 3, Kf]."""
    x = theta0.copy()
    ends = []
    for _ in range(nsteps):
        th, fe, fi = sdc.spread(lv_f, x, sd_f.M + 1, linear_coriolis)
        for _ in range(n_iter):
            th, fe, fi = iteration(lv_f, lv_c, sd_f, sd_c, dt, th, fe, fi, linear_coriolis)
        x = th[-1].copy()
        ends.append(x.copy())
    return np.array(ends)
