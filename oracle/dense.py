"""Dense references on tiny grids (oracle; test infrastructure only).

synthesis_matrix  S_{i,(l,m)} = Y_l^m(pixel i), all -l <= m <= l <= lmax
                  (the S of eqs. synthesis / uzawa, Sec. 2.2).
analyze_dense     O_dense: the least-squares solution of S a = f (the limit of
                  the HEALPix iteration, eq. richardson, Sec. 2.2); recovers
                  band-limited coefficients exactly when S has full column rank.
richardson_radius_readings
                  eigenvalue readings of I - (4 pi / N) S* S for Table 1.

Parity pinned by: Table 1 (printed values, reproduced as
lambda_max((4 pi/N) S* S) - 1 with lmax = 2 Nside), exact recovery of
band-limited coefficients.
"""

import numpy as np

from .geometry import pixel_angles
from .legendre import plm_orthonormal


def synthesis_matrix(nside, lmax):
    """Complex N x (lmax+1)^2 matrix; column order (l, m) with m = -l..l."""
    theta, lam = pixel_angles(nside)
    z = np.cos(theta)
    uz, inv = np.unique(z, return_inverse=True)
    cols = []
    # Pt_l^m at the distinct ring heights
    P = {m: plm_orthonormal(lmax, m, uz) for m in range(lmax + 1)}
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            y = P[am][l - am][inv] * np.exp(1j * am * lam) / np.sqrt(2.0 * np.pi)
            if m < 0:
                y = (-1) ** am * np.conj(y)
            cols.append(y)
    return np.stack(cols, axis=1)


def analyze_dense(f, nside, lmax):
    """Least-squares a (all m), returned as a[l, m + lmax]."""
    S = synthesis_matrix(nside, lmax)
    sol, *_ = np.linalg.lstsq(S, np.asarray(f, dtype=np.complex128), rcond=None)
    out = np.zeros((lmax + 1, 2 * lmax + 1), dtype=np.complex128)
    i = 0
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            out[l, m + lmax] = sol[i]
            i += 1
    return out


def richardson_radius_readings(nside, lmax):
    """(lambda_max - 1, 1 - lambda_min) of (4 pi / N) S* S."""
    S = synthesis_matrix(nside, lmax)
    N = S.shape[0]
    M = (4.0 * np.pi / N) * (S.conj().T @ S)
    ev = np.linalg.eigvalsh(M)
    return ev[-1] - 1.0, 1.0 - ev[0]
