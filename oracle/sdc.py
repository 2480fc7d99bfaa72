"""IMEX spectral deferred corrections (oracle; test infrastructure).

Sec. 5.1.1: [t^n, t^n + dt] is split by M+1 Gauss-Lobatto nodes
(eq. time_discretization_sdc_nodes).  One sweep applies, for m = 0..M-1,
(eq. update_equation_sdcq_discrete_form, and with tau the FAS form
eq. modified_update_equation_sdcq_discrete_form of Sec. 5.1.2):

  Theta^{m+1,(k+1)} = Theta^n
      + dt sum_{j=1}^{m}   qE_{m+1,j} [F_E(Theta^{j,(k+1)}) - F_E(Theta^{j,(k)})]
      + dt sum_{j=1}^{m+1} qI_{m+1,j} [F_I(Theta^{j,(k+1)}) - F_I(Theta^{j,(k)})]
      + dt sum_{j=0}^{M}   q_{m+1,j}  F(Theta^{j,(k)})  + tau^{m+1}

The j = m+1 implicit term makes each node an implicit system
(I - dt qI_{m+1,m+1} F_I) Theta^{m+1} = b (Sec. 5.4).

Readings (the paper states them loosely or not at all):
  * q_{m+1,j} are the integration weights of the Lagrange interpolant through
    the nodes over [t^n, t^{m+1}] (the text says "quadrature points");
  * qE is forward Euler: qE_{i,j} = tau_{j+1} - tau_j for j < i;
  * qI is U^T from the LU factorization without pivoting of Q^T restricted to
    nodes 1..M (Q has a zero row for node 0, so the full Q^T is singular);
    the node-0 column of qI is zero;
  * F at node 0 is the value stored with the node-0 state (it is evaluated at
    the current initial condition by the caller).
The collocation problem A(Theta) = 1 (x) Theta^n with
A(Theta) = Theta - dt (Q (x) I) F(Theta) (eq. collocation_problem) is the
fixed point; its residual is r^m = Theta^n + dt (Q F)_m + tau_m - Theta^m.
"""

import numpy as np
from numpy.polynomial import polynomial as npoly
from numpy.polynomial import legendre as nleg

from . import swe


def lobatto_nodes(nnodes):
    """Gauss-Lobatto nodes on [0, 1]: 0, the roots of P'_{nnodes-1}, 1."""
    if nnodes < 2:
        raise ValueError("need at least 2 Lobatto nodes")
    M = nnodes - 1
    c = np.zeros(M + 1)
    c[M] = 1.0
    inner = np.sort(nleg.legroots(nleg.legder(c))) if M > 1 else np.array([])
    x = np.concatenate(([-1.0], inner, [1.0]))
    return (x + 1.0) / 2.0


def lagrange_basis(nodes, j):
    """Coefficients (increasing powers) of the Lagrange polynomial l_j."""
    coef = np.array([1.0])
    for i, t in enumerate(nodes):
        if i != j:
            coef = npoly.polymul(coef, np.array([-t, 1.0]) / (nodes[j] - t))
    return coef


def lagrange_matrix(src_nodes, dst_nodes):
    """Pi_ij = l_j^{src}(dst_i): interpolation from src to dst nodes."""
    out = np.zeros((len(dst_nodes), len(src_nodes)))
    for j in range(len(src_nodes)):
        out[:, j] = npoly.polyval(dst_nodes, lagrange_basis(src_nodes, j))
    return out


def q_matrix(nodes):
    """Q_ij = int_0^{tau_i} l_j(s) ds (row 0 is zero, last row = Lobatto weights)."""
    n = len(nodes)
    Q = np.zeros((n, n))
    for j in range(n):
        prim = npoly.polyint(lagrange_basis(nodes, j))
        Q[:, j] = npoly.polyval(nodes, prim) - npoly.polyval(0.0, prim)
    return Q


def qe_matrix(nodes):
    n = len(nodes)
    QE = np.zeros((n, n))
    for i in range(n):
        for j in range(i):
            QE[i, j] = nodes[j + 1] - nodes[j]
    return QE


def qi_matrix(nodes):
    """U^T of the LU (no pivoting) of Q[1:,1:]^T, embedded with zero row/col 0."""
    Q = q_matrix(nodes)
    A = Q[1:, 1:].T.copy()
    n = A.shape[0]
    U = A.copy()
    for k in range(n):
        for i in range(k + 1, n):
            f = U[i, k] / U[k, k]
            U[i, k:] -= f * U[k, k:]
    QI = np.zeros_like(Q)
    QI[1:, 1:] = U.T
    return QI


class SDC:
    """Node set and the three matrices for M+1 Lobatto nodes."""

    def __init__(self, nnodes):
        self.nodes = lobatto_nodes(nnodes)
        self.M = nnodes - 1
        self.Q = q_matrix(self.nodes)
        self.QE = qe_matrix(self.nodes)
        self.QI = qi_matrix(self.nodes)


def spread(lv, theta0, nnodes, linear_coriolis=False):
    """Initial iterate: Theta^0 and F(Theta^0) copied to every node."""
    fe, fi = swe.rhs(lv, theta0, linear_coriolis)
    th = np.repeat(theta0[None], nnodes, axis=0)
    return th, np.repeat(fe[None], nnodes, axis=0), np.repeat(fi[None], nnodes, axis=0)


def sweep(lv, sd, dt, theta, fe, fi, tau=None, linear_coriolis=False, misdc=False):
    """One IMEX SDC sweep.  theta/fe/fi: [M+1, 3, K]; node 0 is the initial
    condition with its F already evaluated.  Returns new (theta, fe, fi).

    misdc: the implicit step of each node in two substeps (Sec. 5.1.1, last
    paragraph; the multi-implicit form of the cited Bourlioux et al. work):
    with F_I = L1 Theta + L2 Theta (physical linear terms, diffusion),
      Theta* = (I - beta L1)^{-1} (b + beta L2 Theta^{m+1,(k)}),
      Theta^{m+1,(k+1)} = (I - beta L2)^{-1} (Theta* - beta L2 Theta^{m+1,(k)}),
    beta = dt qI_{m+1,m+1}: each substep is implicit in its own part, and the
    old value of the other part stands in for it, so the fixed point is the
    same collocation solution."""
    M = sd.M
    th_new, fe_new, fi_new = theta.copy(), fe.copy(), fi.copy()
    ftot = fe + fi
    for m in range(M):
        b = theta[0].copy()
        for j in range(1, m + 1):
            b += dt * sd.QE[m + 1, j] * (fe_new[j] - fe[j])
        for j in range(1, m + 1):
            b += dt * sd.QI[m + 1, j] * (fi_new[j] - fi[j])
        b -= dt * sd.QI[m + 1, m + 1] * fi[m + 1]
        for j in range(M + 1):
            b += dt * sd.Q[m + 1, j] * ftot[j]
        if tau is not None:
            b += tau[m + 1]
        beta = dt * sd.QI[m + 1, m + 1]
        if misdc:
            f2_old = swe.diffusion_rhs(lv, theta[m + 1])
            x_star = swe.gravity_solve(lv, beta, b + beta * f2_old)
            x = swe.diffusion_solve(lv, beta, x_star - beta * f2_old)
        else:
            x = swe.implicit_solve(lv, beta, b)
        th_new[m + 1] = x
        fi_new[m + 1] = swe.implicit_rhs(lv, x)
        fe_new[m + 1] = swe.explicit_rhs(lv, x, linear_coriolis)
    return th_new, fe_new, fi_new


def integral(sd, dt, fe, fi):
    """dt (Q (x) I) F: the node-to-start integrals [M+1, 3, K]."""
    ftot = fe + fi
    return dt * np.einsum("ij,j...->i...", sd.Q, ftot)


def residual(sd, dt, theta, fe, fi, tau=None):
    """r^m = Theta^0 + dt (Q F)_m + tau_m - Theta^m for m = 0..M."""
    r = theta[0][None] + integral(sd, dt, fe, fi) - theta
    if tau is not None:
        r = r + tau
    return r


def residual_norm(sd, dt, theta, fe, fi, tau=None):
    """Per variable max over nodes and modes of |r| -> array [3]."""
    r = residual(sd, dt, theta, fe, fi, tau)
    return np.abs(r).max(axis=(0, 2))


def serial_sdc(lv, sd, dt, theta0, nsteps, nsweeps, linear_coriolis=False, misdc=False):
    """SDC(M+1, N_S) time stepping (spread guess, N_S sweeps per step)."""
    th0 = theta0.copy()
    for _ in range(nsteps):
        th, fe, fi = spread(lv, th0, sd.M + 1, linear_coriolis)
        for _ in range(nsweeps):
            th, fe, fi = sweep(lv, sd, dt, th, fe, fi, None, linear_coriolis, misdc)
        th0 = th[-1].copy()
    return th0
