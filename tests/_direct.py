"""Brute-force evaluation of spherical-harmonic expansions at arbitrary points.

Independent of the oracle's tables and quadrature: the normalized associated
Legendre function comes from scipy.special.lpmv (with its Condon-Shortley
phase removed and the factor sqrt((2n+1)/2 (n-m)!/(n+m)!) applied), and sums
are taken term by term.  Only for tiny truncations.
"""

import math

import numpy as np
from scipy.special import lpmv


def pnm(n, m, mu):
    norm = math.sqrt((2 * n + 1) / 2.0 * math.factorial(n - m) / math.factorial(n + m))
    return norm * (-1) ** m * lpmv(m, n, mu)


def evaluate(spec, T, lam, phi):
    """sum over m=-T..T, n>=|m| of xi_n^m P_n^|m|(sin phi) e^{i m lam} (real field)."""
    mu = np.sin(phi)
    out = np.zeros(np.broadcast(lam, phi).shape)
    k = 0
    for m in range(T + 1):
        for n in range(m, T + 1):
            c = spec[k]
            k += 1
            if c == 0:
                continue
            term = c * pnm(n, m, mu) * np.exp(1j * m * lam)
            out = out + (term.real if m == 0 else 2.0 * term.real)
    return out
