"""Rotating shallow-water operators in the SH basis (oracle; test infrastructure).

Sec. 2: prognostic U = [Phi, zeta, delta]; dU/dt = L(U) + N(U) with
  L = [ -Phibar delta + nu lap Phi',  nu lap zeta,  -lap Phi + nu lap delta ]
      (eq. linear_wave_motion_induced_by_gravitational_forces)
  N = [ -div(Phi' V),  -div((zeta+f) V),  k.curl((zeta+f) V) - lap(V.V/2) ]
      (eq. nonlinear_operators), f = 2 Omega sin(phi),
and the Helmholtz split V = k x grad psi + grad chi, zeta = lap psi,
delta = lap chi (eq. helmholtz_theorem).
Sec. 4: F_I = L (implicit), F_E = N (explicit).
Sec. 5.4: the implicit systems (I - dt qI_{m+1,m+1} F_I) Theta = b are solved by
local (per-mode) updates.

The nonlinear terms are evaluated with the transform method: U = u cos(phi) and
V = v cos(phi) are synthesized from psi and chi with P and H = (1-mu^2) dP/dmu,
the products A = eta U, B = eta V, C = Phi' U, D = Phi' V,
E = (U^2+V^2)/(2(1-mu^2)) are formed on the grid (eta = zeta + 2 Omega mu), and
the divergence/curl are returned to spectral space with the quadrature form
(integration by parts in mu):
  D[X,Y]_n^m = sum_j w_j/(a(1-mu_j^2)) [ i m X_m(mu_j) P_n^m(mu_j) - Y_m(mu_j) H_n^m(mu_j) ]
  N_zeta = -D[A,B],  N_delta = D[B,-A] + n(n+1)/a^2 sum_j w_j P_n^m E_m,  N_Phi = -D[C,D].

State layout: complex128 array [3, K] with variable order (Phi, zeta, delta),
m-major spectral layout of ``sht``.
"""

from dataclasses import dataclass

import numpy as np

from . import sht


@dataclass
class Physics:
    radius: float = 6.371e6
    omega: float = 7.292e-5
    phibar: float = 9.81 * 1e4
    nu: float = 1e5


class Level:
    """One spatial level: grid, tables and the physical constants."""

    def __init__(self, T, nlat, nlon, phys=None):
        self.g = sht.Grid(T, nlat, nlon)
        self.phys = phys if phys is not None else Physics()
        self.T, self.K = T, self.g.K
        n = self.g.n_of.astype(np.float64)
        a = self.phys.radius
        self.lam = -n * (n + 1) / (a * a)          # eigenvalues of lap
        self.nn1 = n * (n + 1)


# --------------------------------------------------------------- linear part
def implicit_rhs(lv, theta):
    """F_I = L(Theta) per mode (lap -> lam_n = -n(n+1)/a^2; lap of the
    constant Phibar is 0, so nu lap Phi' = nu lam Phi)."""
    p = lv.phys
    phi, zeta, delta = theta
    lam = lv.lam
    out = np.empty_like(theta)
    out[0] = -p.phibar * delta + p.nu * lam * phi
    out[1] = p.nu * lam * zeta
    out[2] = -lam * phi + p.nu * lam * delta
    return out


def implicit_solve(lv, beta, b):
    """Solve (I - beta L) x = b mode by mode (Sec. 5.4).

    zeta:         d zeta = b_zeta,                   d = 1 - beta nu lam
    (Phi, delta): [[d, beta Phibar], [beta lam, d]] [Phi, delta] = [b_Phi, b_delta]
    """
    p = lv.phys
    lam = lv.lam
    d = 1.0 - beta * p.nu * lam
    det = d * d - beta * beta * p.phibar * lam
    x = np.empty_like(b)
    x[1] = b[1] / d
    x[0] = (d * b[0] - beta * p.phibar * b[2]) / det
    x[2] = (d * b[2] - beta * lam * b[0]) / det
    return x


# The two parts of L for the two-substep (multi-implicit) variant of the
# implicit step (Sec. 5.1.1, last paragraph): L = L1 + L2 with L1 the physical
# linear terms (gravity waves) and L2 the artificial diffusion nu lap.
def gravity_rhs(lv, theta):
    """L1 Theta: (-Phibar delta, 0, -lam Phi) per mode."""
    p = lv.phys
    out = np.zeros_like(theta)
    out[0] = -p.phibar * theta[2]
    out[2] = -lv.lam * theta[0]
    return out


def diffusion_rhs(lv, theta):
    """L2 Theta = nu lam_n Theta per mode and variable."""
    return lv.phys.nu * lv.lam * theta


def gravity_solve(lv, beta, b):
    """Solve (I - beta L1) x = b: zeta unchanged, a 2x2 system for (Phi, delta)
    with det = 1 - beta^2 Phibar lam."""
    p = lv.phys
    lam = lv.lam
    det = 1.0 - beta * beta * p.phibar * lam
    x = np.empty_like(b)
    x[1] = b[1]
    x[0] = (b[0] - beta * p.phibar * b[2]) / det
    x[2] = (b[2] - beta * lam * b[0]) / det
    return x


def diffusion_solve(lv, beta, b):
    """Solve (I - beta L2) x = b: x = b / (1 - beta nu lam) per mode."""
    return b / (1.0 - beta * lv.phys.nu * lv.lam)


# ------------------------------------------------------------ nonlinear part
def streamfunction(lv, field):
    """psi = lap^{-1} zeta (likewise chi from delta): -a^2/(n(n+1)) per mode, 0 at n=0."""
    out = np.zeros_like(field)
    nz = lv.nn1 > 0
    out[nz] = -(lv.phys.radius ** 2) / lv.nn1[nz] * field[nz]
    return out


def uv_fourier(lv, psi, chi):
    """Fourier coefficients of U = u cos(phi), V = v cos(phi):
    U_m = (1/a) sum_n [ i m chi_n P_n - psi_n H_n ],
    V_m = (1/a) sum_n [ i m psi_n P_n + chi_n H_n ]."""
    g, T, a = lv.g, lv.T, lv.phys.radius
    U = np.zeros((g.nlat, T + 1), dtype=np.complex128)
    V = np.zeros((g.nlat, T + 1), dtype=np.complex128)
    for m in range(T + 1):
        o = sht.offset(T, m)
        sl = slice(o, o + T + 1 - m)
        P = g.P[m][: T + 1 - m]
        H = g.H[m]
        U[:, m] = (1j * m * chi[sl] @ P - psi[sl] @ H) / a
        V[:, m] = (1j * m * psi[sl] @ P + chi[sl] @ H) / a
    return U, V


def _div_form(lv, X, Y):
    """D[X,Y]_n^m = sum_j w_j/(a(1-mu_j^2)) [ i m X_m P_n^m - Y_m H_n^m ]."""
    g, T, a = lv.g, lv.T, lv.phys.radius
    wt = g.w / (a * (1.0 - g.mu ** 2))
    out = np.zeros(lv.K, dtype=np.complex128)
    for m in range(T + 1):
        o = sht.offset(T, m)
        P = g.P[m][: T + 1 - m]
        H = g.H[m]
        out[o:o + T + 1 - m] = 1j * m * (P @ (wt * X[:, m])) - H @ (wt * Y[:, m])
    return out


def explicit_rhs(lv, theta, linear_coriolis=False):
    """F_E = N(Theta) by the transform method.

    linear_coriolis=True keeps only the terms linear in the state with the
    Coriolis parameter (A = f U, B = f V, C = D = E = 0); it is a test-only
    flag that turns the system into a linear ODE with a matrix exponential."""
    g, p = lv.g, lv.phys
    phi, zeta, delta = theta
    psi = streamfunction(lv, zeta)
    chi = streamfunction(lv, delta)
    Uf, Vf = uv_fourier(lv, psi, chi)
    U = sht.fourier_synthesis(g, Uf)
    V = sht.fourier_synthesis(g, Vf)
    phip = phi.copy()
    phip[0] = phip[0] - np.sqrt(2.0) * p.phibar     # Phi' = Phi - Phibar (P_0^0 = 1/sqrt 2)
    Phi_g = sht.synthesis(g, phip)
    zeta_g = sht.synthesis(g, zeta)
    f = 2.0 * p.omega * g.mu[:, None]
    if linear_coriolis:
        eta = f + 0.0 * zeta_g
        Phi_g = 0.0 * Phi_g
        kin = 0.0 * U
    else:
        eta = zeta_g + f
        kin = (U * U + V * V) / (2.0 * (1.0 - g.mu[:, None] ** 2))
    A = sht.fourier_analysis(g, eta * U)
    B = sht.fourier_analysis(g, eta * V)
    C = sht.fourier_analysis(g, Phi_g * U)
    D = sht.fourier_analysis(g, Phi_g * V)
    E = sht.legendre_analysis(g, sht.fourier_analysis(g, kin))
    out = np.empty_like(theta)
    out[0] = -_div_form(lv, C, D)
    out[1] = -_div_form(lv, A, B)
    out[2] = _div_form(lv, B, -A) + lv.nn1 / p.radius ** 2 * E
    for k in range(3):
        out[k][: lv.T + 1] = out[k][: lv.T + 1].real     # Im of m = 0 is 0
    return out


def rhs(lv, theta, linear_coriolis=False):
    """(F_E, F_I) at one state."""
    return explicit_rhs(lv, theta, linear_coriolis), implicit_rhs(lv, theta)
