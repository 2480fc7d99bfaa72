"""Pin of the error norm of Sec. 6 (eq. error_norm_r_norm) on hand-made cases."""

import numpy as np

from oracle import metrics, sht


def test_error_norm_hand_cases():
    T = 8
    ref = np.zeros(sht.ncoef(T), dtype=np.complex128)
    ref[sht.index(T, 0, 0)] = 100.0
    ref[sht.index(T, 1, 3)] = 2.0
    ref[sht.index(T, 5, 7)] = 4.0
    phi = ref.copy()
    phi[sht.index(T, 5, 7)] += 0.5j          # error only at n = 7
    assert metrics.error_norm(phi, ref, T) == 0.5 / 100.0
    assert metrics.error_norm(phi, ref, T, exclude_mean=True) == 0.5 / 4.0
    assert metrics.error_norm(phi, ref, T, R_norm=6) == 0.0   # outside the semi-norm
    phi[sht.index(T, 1, 3)] += 1.0
    assert metrics.error_norm(phi, ref, T, R_norm=3, exclude_mean=True) == 1.0 / 2.0
