"""Seeded synthetic initial states shared by tests, bench and smoke.

This module only draws numbers and places closed-form initial-condition
coefficients; it holds none of the transform, operator or time-stepping
arithmetic, so both the GPU library and the CPU oracle can be fed from it.

Layout: complex128 [3, K] per state (Phi, zeta, delta), spectral m-major
(m = 0..T, n = m..T), K = (T+1)(T+2)/2, normalized Legendre functions with
P_0^0 = 1/sqrt(2), P_1^0 = sqrt(3/2) mu, P_2^0 = sqrt(5/2) (3 mu^2 - 1)/2.

Recipe (stands in for the paper's test cases, whose fields are "rapidly
decaying modes across the full spectrum"):
  * random part: coefficient = A_var * z * n^-p for 1 <= n <= T, z complex
    normal (x + i y)/sqrt(2), real normal for m = 0; A_Phi = 1e3 m^2/s^2,
    A_zeta = 1e-5 1/s, A_delta = 1e-6 1/s; n = 0 is zero for zeta and delta;
    draws are made in the order Phi, zeta, delta, each m-major;
  * mean geopotential: Phi_0^0 = sqrt(2) Phibar;
  * balanced zonal solid-body flow u = u0 cos(phi): zeta_1^0 += (2 u0/a) sqrt(2/3),
    Phi += -(a Omega u0 + u0^2/2)(mu^2 - 1/3), i.e. Phi_2^0 += -(a Omega u0 + u0^2/2)(2/3) sqrt(2/5).
"""

import numpy as np

RADIUS = 6.371e6
OMEGA = 7.292e-5
PHIBAR = 9.81 * 1e4
NU = 1e5
AMPLITUDES = (1e3, 1e-5, 1e-6)


def ncoef(T):
    return (T + 1) * (T + 2) // 2


def _mn(T):
    m = np.concatenate([np.full(T + 1 - mm, mm) for mm in range(T + 1)])
    n = np.concatenate([np.arange(mm, T + 1) for mm in range(T + 1)])
    return m, n


def _slot(T, m, n):
    return m * (T + 1) - m * (m - 1) // 2 + (n - m)


def random_spectrum(T, seed, power=2.0, amplitudes=AMPLITUDES):
    rng = np.random.default_rng(seed)
    K = ncoef(T)
    m, n = _mn(T)
    x = rng.standard_normal((3, K))
    y = rng.standard_normal((3, K))
    z = np.where(m[None, :] == 0, x + 0j, (x + 1j * y) / np.sqrt(2.0))
    scale = np.zeros(K)
    scale[n >= 1] = n[n >= 1].astype(np.float64) ** (-power)
    out = z * scale[None, :] * np.asarray(amplitudes)[:, None]
    return out.astype(np.complex128)


def mean_geopotential(T, phibar=PHIBAR):
    out = np.zeros((3, ncoef(T)), dtype=np.complex128)
    out[0, 0] = np.sqrt(2.0) * phibar
    return out


def solid_body(T, u0=20.0, radius=RADIUS, omega=OMEGA):
    out = np.zeros((3, ncoef(T)), dtype=np.complex128)
    out[1, _slot(T, 0, 1)] = (2.0 * u0 / radius) * np.sqrt(2.0 / 3.0)
    if T >= 2:
        out[0, _slot(T, 0, 2)] = -(radius * omega * u0 + 0.5 * u0 * u0) * (2.0 / 3.0) * np.sqrt(2.0 / 5.0)
    return out


def seeded_state(T, seed, power=2.0, u0=20.0, phibar=PHIBAR):
    """Random n^-power spectra + mean geopotential + balanced solid body."""
    return random_spectrum(T, seed, power) + mean_geopotential(T, phibar) + solid_body(T, u0)


def seeded_batch(T, seeds, power=2.0, u0=20.0):
    return np.stack([seeded_state(T, s, power, u0) for s in seeds])
