"""O_synth: exact spherical-harmonic synthesis on the HEALPix points (oracle).

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

Eq. (synthesis), Sec. 2.2: f_i = sum_{l <= lmax} sum_{|m| <= l} a_l^m Y_l^m(pixel i).
For a real map a_l^{-m} = (-1)^m conj(a_l^m), so with the packed m >= 0
coefficients
   f(lambda, theta_r) = Re sum_{m >= 0} w_m F_m(theta_r) e^{i m lambda},
   F_m(theta) = sum_l a_l^m Pt_l^m(cos theta) / sqrt(2 pi),  w_0 = 1, w_m = 2.
F_m is a direct Legendre sum per ring; the longitude sum at the n points of
a ring, lambda_q = phi0 + 2 pi q / n, folds m onto m mod n and uses an inverse
FFT of length n (exact: e^{i m lambda_q} depends on m only through m mod n
once the phase e^{i m phi0} is applied).  Rings r and 4 Nside - r share |z|,
and Pt_l^m(-z) = (-1)^{l+m} Pt_l^m(z), so the Legendre sums are taken on the
northern rings and the equator only.

Parity pinned by: synthesis of single harmonics against scipy's
sph_harm_y at the pixel centres, and O_dense(O_synth(a)) = a (exact recovery
of band-limited coefficients, P6).
"""

import numpy as np

from .geometry import ring_table
from .legendre import plm_rows


def synthesize(alm, nside, lmax):
    alm = np.asarray(alm, dtype=np.complex128)
    if alm.size != (lmax + 1) * (lmax + 2) // 2:
        raise ValueError("alm has the wrong size for lmax")
    rt = ring_table(nside)
    nr = len(rt["n"])
    half = 2 * nside                       # rings 1 .. 2 Nside (north + equator)
    zn = rt["z"][:half]
    Fn = np.zeros((lmax + 1, half), dtype=np.complex128)   # F_m on northern rings
    Fs = np.zeros((lmax + 1, half), dtype=np.complex128)   # F_m on mirrored rings
    ms = np.arange(lmax + 1)
    base = ms * (2 * lmax + 1 - ms) // 2
    for l, P in plm_rows(lmax, zn):
        a_l = alm[base[:l + 1] + l]                        # a_l^m, m = 0 .. l
        contrib = a_l[:, None] * P                          # (m, ring)
        Fn[:l + 1] += contrib
        par = (-1.0) ** (l + ms[:l + 1])
        Fs[:l + 1] += par[:, None] * contrib
    Fn /= np.sqrt(2.0 * np.pi)
    Fs /= np.sqrt(2.0 * np.pi)
    out = np.empty(int(np.sum(rt["n"])))
    w = np.where(ms == 0, 1.0, 2.0)
    for r in range(nr):
        if r < half:
            F = Fn[:, r]
        else:
            F = Fs[:, nr - 1 - r]
        n = int(rt["n"][r])
        spec = np.zeros(n, dtype=np.complex128)
        np.add.at(spec, ms % n, w * F * np.exp(1j * ms * rt["phi0"][r]))
        vals = np.fft.ifft(spec) * n
        out[rt["start"][r]:rt["start"][r] + n] = vals.real
    return out
