"""Equal-weight (HEALPix-style) analysis and its Jacobi iteration (oracle).

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

analyze_equal_weight   eq. (healsph), Sec. 2.2:
    a_l^m = (4 pi / N) sum_i conj(Y_l^m(pixel i)) f_i,   0 <= m <= l <= lmax,
    i.e. a = A f with A = (4 pi / N) S^* (the equal-weight quadrature of the
    inner product, eq. sphip).  Pixels of one ring share theta, so with the
    longitude sum of ring r
        F_r(m) = sum_q f_q e^{-i m lambda_q},  lambda_q = phi0_r + 2 pi q / n_r,
    taken for every m <= lmax (no truncation at the ring's Nyquist mode: the
    sum itself repeats with period n_r in m), the coefficient is
        a_l^m = (4 pi / N) sum_r Pt_l^m(z_r) F_r(m) / sqrt(2 pi).
    F_r(m) = e^{-i m phi0_r} DFT(f_r)[m mod n_r] with numpy's FFT as the step.

analyze_jacobi         eq. (uzawa), Sec. 2.2, with A = (4 pi / N) S^* and the
    exact synthesis S (O_synth):
        a^(0) = A f,   a^(k+1) = a^(k) + A (f - S a^(k)),
    which is Richardson iteration on the normal equations, eq. (richardson).

Parity pinned by (tests/test_oracle_healpix.py): the dense route
(4 pi / N) S^H f with the synthesis matrix of dense.py (itself pinned by the
printed Table 1) for lmax below and above 2 Nside; the constant map
(a_0^0 = sqrt(4 pi) c, orders not divisible by 4 vanish by the quarter-turn
symmetry of the grid); the error contraction of the iteration on band-limited
input, bounded by the printed spectral radii of Table 1; and the fixed point
of the iteration, the least-squares solution O_dense.
"""

import numpy as np

from .geometry import ring_table
from .legendre import plm_rows


def ring_longitude_sums(f, nside, lmax):
    """F[r, m] = sum_q f_q e^{-i m lambda_q} for every ring r, m = 0..lmax."""
    rt = ring_table(nside)
    f = np.asarray(f, dtype=np.float64)
    ms = np.arange(lmax + 1)
    F = np.empty((len(rt["n"]), lmax + 1), dtype=np.complex128)
    for r in range(len(rt["n"])):
        n = int(rt["n"][r])
        s = int(rt["start"][r])
        dft = np.fft.fft(f[s:s + n])                 # sum_q f_q e^{-2 pi i q k / n}
        F[r] = np.exp(-1j * ms * rt["phi0"][r]) * dft[ms % n]
    return F


def analyze_equal_weight(f, nside, lmax):
    """Packed a_l^m (m >= 0, index m (2 lmax + 1 - m) / 2 + l) of eq. (healsph)."""
    rt = ring_table(nside)
    N = int(np.sum(rt["n"]))
    F = ring_longitude_sums(f, nside, lmax)          # (ring, m)
    ms = np.arange(lmax + 1)
    base = ms * (2 * lmax + 1 - ms) // 2
    out = np.zeros((lmax + 1) * (lmax + 2) // 2, dtype=np.complex128)
    scale = 4.0 * np.pi / N / np.sqrt(2.0 * np.pi)
    for l, P in plm_rows(lmax, rt["z"]):            # P[m, r] = Pt_l^m(z_r), m <= l
        out[base[:l + 1] + l] = scale * np.einsum("mr,rm->m", P, F[:, :l + 1])
    return out


def analyze_jacobi(f, nside, lmax, niter):
    """a^(niter) of eq. (uzawa) with A = (4 pi / N) S^* (niter = 0: plain A f)."""
    from .synth import synthesize
    f = np.asarray(f, dtype=np.float64)
    a = analyze_equal_weight(f, nside, lmax)
    for _ in range(int(niter)):
        a = a + analyze_equal_weight(f - synthesize(a, nside, lmax), nside, lmax)
    return a


def equal_weight_columns(f, nside, ms, lmax):
    """{m: a_l^m for l = m..lmax} of eq. (healsph) for the listed orders only
    (the same sums, with the order-m Legendre functions evaluated directly at
    the ring heights): affordable at large nside for a few orders."""
    from .legendre import plm_orthonormal
    rt = ring_table(nside)
    N = int(np.sum(rt["n"]))
    F = ring_longitude_sums(f, nside, lmax)
    scale = 4.0 * np.pi / N / np.sqrt(2.0 * np.pi)
    out = {}
    for m in ms:
        P = plm_orthonormal(lmax, int(m), rt["z"])    # [l - m][ring]
        out[int(m)] = scale * (P @ F[:, int(m)])
    return out
