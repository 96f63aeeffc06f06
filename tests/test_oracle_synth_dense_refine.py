"""Pins of O_synth, O_dense, the power spectrum and O_ref (CPU only)."""

import numpy as np
import pytest
import scipy.special as sp

import oracle as O
from oracle.geometry import pixel_angles
from oracle.legendre import gauss_legendre, ylm
from oracle.spectrum import alm_index, alm_size
import workloads as W


def _rand_alm(lmax, seed, with_low=True):
    rng = np.random.default_rng(seed)
    a = (rng.standard_normal(alm_size(lmax)) + 1j * rng.standard_normal(alm_size(lmax)))
    for l in range(lmax + 1):
        a[alm_index(l, 0, lmax)] = a[alm_index(l, 0, lmax)].real
    return a


def _full_from_packed(a, lmax):
    full = np.zeros((lmax + 1, 2 * lmax + 1), dtype=np.complex128)
    for l in range(lmax + 1):
        for m in range(l + 1):
            v = a[alm_index(l, m, lmax)]
            full[l, lmax + m] = v
            full[l, lmax - m] = (-1) ** m * np.conj(v)
    return full


@pytest.mark.parametrize("l,m", [(0, 0), (3, 0), (5, 2), (12, 11), (16, 16)])
def test_synthesis_of_single_harmonic_matches_scipy(l, m):
    nside, lmax = 8, 16
    a = np.zeros(alm_size(lmax), dtype=np.complex128)
    val = 0.7 - 0.3j if m else 0.7
    a[alm_index(l, m, lmax)] = val
    f = O.synthesize(a, nside, lmax)
    th, lam = pixel_angles(nside)
    y = sp.sph_harm_y(l, m, th, lam)
    ref = (val * y).real if m == 0 else 2.0 * (val * y).real
    assert np.max(np.abs(f - ref)) < 1e-13


@pytest.mark.parametrize("nside", [2, 4, 8])
def test_dense_least_squares_recovers_band_limited_coefficients(nside):
    lmax = 2 * nside
    a = _rand_alm(lmax, 10 + nside)
    f = O.synthesize(a, nside, lmax)
    ad = O.analyze_dense(f, nside, lmax)
    assert np.max(np.abs(ad - _full_from_packed(a, lmax))) < 1e-11


def test_parseval_against_independent_quadrature():
    """sum_l (2l+1) C_l = int |f|^2 dOmega, the integral by Gauss-Legendre x
    equispaced quadrature of f evaluated with scipy's spherical harmonics."""
    lmax = 10
    a = _rand_alm(lmax, 3)
    x, w = gauss_legendre(lmax + 2)
    nphi = 2 * lmax + 2
    th = np.arccos(x)[:, None] * np.ones((1, nphi))
    ph = np.ones((len(x), 1)) * (2 * np.pi * np.arange(nphi) / nphi)[None, :]
    f = np.zeros_like(th)
    for l in range(lmax + 1):
        for m in range(l + 1):
            y = sp.sph_harm_y(l, m, th, ph)
            v = a[alm_index(l, m, lmax)]
            f += (v * y).real if m == 0 else 2.0 * (v * y).real
    integral = np.sum(w[:, None] * f * f) * (2 * np.pi / nphi)
    cl = O.power_spectrum(a, lmax)
    assert np.sum((2 * np.arange(lmax + 1) + 1) * cl) == pytest.approx(integral, rel=1e-12)


def test_power_spectrum_counts_negative_orders_once_each():
    lmax = 3
    a = np.zeros(alm_size(lmax), dtype=np.complex128)
    a[alm_index(3, 0, lmax)] = 2.0
    a[alm_index(3, 2, lmax)] = 1.0 + 1.0j
    cl = O.power_spectrum(a, lmax)
    assert cl[3] == pytest.approx((4.0 + 2 * 2.0) / 7.0)
    assert cl[0] == cl[1] == cl[2] == 0.0


def test_hp2sph_method_error_on_band_limited_input_is_recorded():
    """Not a pin: HP2SPH is not exact for band-limited input (polar aliasing);
    its distance from the dense least-squares solution is measured and must
    be small for a decaying spectrum."""
    nside = 16
    lmax = 2 * nside
    rng = W.rng_for(0, 0)
    a = W.draw_alm(W.spectrum(0, lmax), lmax, rng)
    f = O.synthesize(a, nside, lmax)
    ah = O.analyze(f, nside, lmax)
    err = np.max(np.abs(ah - a)) / np.max(np.abs(a))
    assert 1e-10 < err < 0.5


def test_refinement_leaves_exactly_recovered_input_unchanged():
    nside = 8
    th, lam = pixel_angles(nside)
    f = ylm(9, 1, th, lam).real + 0.3 * ylm(2, 0, th, lam).real
    a0 = O.analyze(f, nside)
    a1 = O.analyze_refined(f, nside)
    assert np.max(np.abs(a1 - a0)) < 1e-13


def test_refinement_does_not_move_away_from_band_limited_truth():
    """Recorded property, not a pin: one round of eq. (uzawa) with A = HP2SPH
    reduces the error on band-limited input only partly, because A S keeps
    the polar-aliased components (A S != I)."""
    nside = 16
    lmax = 2 * nside
    rng = W.rng_for(0, 1)
    a = W.draw_alm(W.spectrum(0, lmax), lmax, rng)
    f = O.synthesize(a, nside, lmax)
    e0 = np.max(np.abs(O.analyze(f, nside) - a))
    e1 = np.max(np.abs(O.analyze_refined(f, nside) - a))
    assert e1 < 0.9 * e0
