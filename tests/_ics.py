"""Initial condition of the zonal-jet workload (test infrastructure).

A balanced zonal jet u = 80 m/s sech^2((phi - 45 deg)/6 deg) plus a 120 m
Gaussian height bump of the dome shape of Sec. 6.1 (centre lambda = pi,
phi = pi/4, width constant alpha = 20), on top of the seeded n^-2 spectra and
the mean geopotential.  Fields are built on the Gaussian grid and brought to
spectral space with the oracle's analysis, so this module is test-only.

Balance (gradient wind, from the divergence equation with the tendency of
delta set to zero for a steady zonal flow): dPhi/dphi = -a u (f + u tan(phi)/a),
integrated from the south pole with a fine trapezoid rule and shifted so that
the Gauss-weighted global mean of Phi is Phibar.
"""

import numpy as np

from oracle import sht, swe
from paper_1904_05988_amd import inputs

G = 9.81


def jet_fields(lv, u0=80.0, phi0=np.deg2rad(45.0), width=np.deg2rad(6.0), bump=120.0,
               alpha=20.0):
    g, p = lv.g, lv.phys
    a, Om = p.radius, p.omega
    phi = np.arcsin(g.mu)
    lam = g.lam

    def u_of(ph):
        return u0 / np.cosh((ph - phi0) / width) ** 2

    def du_of(ph):
        s = (ph - phi0) / width
        return -2.0 * u0 / np.cosh(s) ** 2 * np.tanh(s) / width

    # zeta = -(1/(a cos phi)) d(u cos phi)/dphi = -u'/a + u tan(phi)/a
    zeta_lat = (-du_of(phi) + u_of(phi) * np.tan(phi)) / a
    # Phi(phi) by integrating the gradient-wind balance
    fine = np.linspace(-np.pi / 2, np.pi / 2, 200001)
    uf = u_of(fine)
    integrand = -a * uf * (2 * Om * np.sin(fine) + uf * np.tan(np.clip(fine, -1.5707, 1.5707)) / a)
    prim = np.concatenate(([0.0], np.cumsum(0.5 * (integrand[1:] + integrand[:-1]) * np.diff(fine))))
    phi_lat = np.interp(phi, fine, prim)
    phi_lat = phi_lat - np.sum(g.w * phi_lat) / 2.0 + p.phibar
    lamg, phig = np.meshgrid(lam, phi)
    x = a * (np.cos(lamg) * np.cos(phig) - np.cos(np.pi) * np.cos(np.pi / 4))
    y = a * (np.sin(lamg) * np.cos(phig) - np.sin(np.pi) * np.cos(np.pi / 4))
    z = a * (np.sin(phig) - np.sin(np.pi / 4))
    d2 = (x * x + y * y + z * z) / (a * a)
    Phi = phi_lat[:, None] + G * bump * np.exp(-alpha * d2)
    Zeta = np.repeat(zeta_lat[:, None], lv.g.nlon, axis=1)
    return Phi, Zeta


def jet_state(T, nlat, nlon, seed):
    lv = swe.Level(T, nlat, nlon)
    Phi, Zeta = jet_fields(lv)
    st = inputs.random_spectrum(T, seed).copy()
    st[0] += sht.analysis(lv.g, Phi)
    st[1] += sht.analysis(lv.g, Zeta)
    return st
