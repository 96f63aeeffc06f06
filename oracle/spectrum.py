"""Angular power spectrum, eq. (APS), Sec. 1 (oracle; test infrastructure only).

C_l = (1/(2l+1)) sum_{m=-l}^{l} |a_l^m|^2; for a real map |a_l^{-m}| = |a_l^m|,
so C_l = (|a_l^0|^2 + 2 sum_{m=1}^{l} |a_l^m|^2) / (2l+1) from the packed
m >= 0 coefficients (layout: index m (2 lmax + 1 - m)/2 + l).

Parity pinned by: Parseval, sum_l (2l+1) C_l = int |f|^2 dOmega, for
band-limited f through O_dense (P10).
"""

import numpy as np


def alm_size(lmax):
    return (lmax + 1) * (lmax + 2) // 2


def alm_index(l, m, lmax):
    return m * (2 * lmax + 1 - m) // 2 + l


def power_spectrum(alm, lmax):
    alm = np.asarray(alm, dtype=np.complex128)
    cl = np.zeros(lmax + 1)
    for m in range(lmax + 1):
        base = m * (2 * lmax + 1 - m) // 2
        v = np.abs(alm[base + m:base + lmax + 1]) ** 2
        cl[m:] += v if m == 0 else 2.0 * v
    return cl / (2.0 * np.arange(lmax + 1) + 1.0)
