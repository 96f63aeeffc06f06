"""Helpers shared by the GPU tests (inputs built on the CPU with the oracle)."""

import numpy as np

import oracle as O
import workloads as W


def cmb_map(config_id, map_index, nside, lmax=None):
    """A seeded CMB-like map (oracle synthesis of Gaussian a_lm), and its a_lm."""
    lmax = 2 * nside if lmax is None else lmax
    rng = W.rng_for(config_id, map_index)
    a = W.draw_alm(W.spectrum(config_id, lmax), lmax, rng)
    return O.synthesize(a, nside, lmax), a


def white_map(nside, seed):
    return W.random_map(O.npix(nside), W.rng_for(99, seed))


def rel_err(x, ref):
    return float(np.max(np.abs(np.asarray(x) - np.asarray(ref))) / max(np.max(np.abs(ref)), 1e-300))


def _ring_z_ld(nside):
    """cos(theta) of every ring from eq. (healpts), in extended precision."""
    ld = np.longdouble
    n = ld(nside)
    nr = 4 * nside - 1
    z = np.empty(nr, dtype=ld)
    for r in range(1, nr + 1):
        if r < nside:
            z[r - 1] = 1 - ld(r) * ld(r) / (3 * n * n)
        elif r <= 3 * nside:
            z[r - 1] = 2 * (2 * n - ld(r)) / (3 * n)
        else:
            j = ld(4 * nside - r)
            z[r - 1] = -(1 - j * j / (3 * n * n))
    return z


def _plm1_ld(lmax, z):
    """Orthonormal Pt_l^1(z), l = 1 .. lmax (Condon-Shortley phase), by the
    three-term recurrence in extended precision, rounded once to double.
    Near the poles dPt_l/dz ~ l^2, so z itself must be exact to ~1e-19."""
    ld = np.longdouble
    s = np.sqrt((1 - z) * (1 + z))
    out = np.empty((lmax, z.size))
    p1 = -np.sqrt(ld(3) / 4) * s
    p2 = np.sqrt(ld(5)) * z * p1
    out[0] = p1.astype(np.float64)
    if lmax >= 2:
        out[1] = p2.astype(np.float64)
    for l in range(3, lmax + 1):
        L = ld(l)
        a = np.sqrt((4 * L * L - 1) / (L * L - 1))
        b = np.sqrt((2 * L + 1) * ((L - 1) * (L - 1) - 1) / ((2 * L - 3) * (L * L - 1)))
        p1, p2 = p2, a * z * p2 - b * p1
        out[l - 1] = p2.astype(np.float64)
    return out


def order_one_fields(nside, batch, config_id):
    """Real fields f = 2 Re(sum_{l=1}^{p} c_l Y_l^1), one per map, seeded c_l
    (complex Gaussian / l), Y_l^1 as in the oracle (Appendix A convention) with
    the Legendre functions evaluated at the exact ring heights in extended
    precision.  HP2SPH recovers these exactly for every l <= p (pinned on the
    oracle).  Returns (maps (batch, npix), expected packed a_lm)."""
    lmax = 2 * nside
    rt = O.ring_table(nside)
    pt = _plm1_ld(lmax, _ring_z_ld(nside))                    # (lmax, rings), l = 1 .. lmax
    l = np.arange(1, lmax + 1)
    coef = np.empty((batch, lmax), dtype=np.complex128)
    for v in range(batch):
        rng = W.rng_for(config_id, v)
        coef[v] = (rng.standard_normal(lmax) + 1j * rng.standard_normal(lmax)) / np.sqrt(2.0) / l
    F = coef @ pt                                              # (batch, rings)
    maps = np.empty((batch, O.npix(nside)))
    for r in range(len(rt["n"])):
        n, s0 = int(rt["n"][r]), int(rt["start"][r])
        lam = rt["phi0"][r] + 2.0 * np.pi * np.arange(n) / n
        maps[:, s0:s0 + n] = 2.0 * np.real(F[:, r:r + 1] * np.exp(1j * lam)[None, :]) / np.sqrt(2.0 * np.pi)
    expect = np.zeros((batch, O.alm_size(lmax)), dtype=np.complex128)
    idx = np.array([O.alm_index(ll, 1, lmax) for ll in range(1, lmax + 1)])
    expect[:, idx] = coef
    return maps, expect
