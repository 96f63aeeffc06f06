"""Pins of the oracle's point set and Legendre functions (CPU only)."""

import numpy as np
import pytest
import scipy.special as sp

from oracle.geometry import ring_table, pixel_angles, npix
from oracle.legendre import plm_orthonormal, plm_rows, ylm, gauss_legendre


@pytest.mark.parametrize("nside", [2, 4, 8, 64, 256])
def test_pixel_and_ring_counts(nside):
    rt = ring_table(nside)
    assert len(rt["n"]) == 4 * nside - 1
    assert int(rt["n"].sum()) == npix(nside) == 12 * nside * nside
    # polar rings carry 4j points, the belt 4 Nside
    assert list(rt["n"][:nside - 1]) == [4 * j for j in range(1, nside)]
    assert np.all(rt["n"][nside - 1:3 * nside] == 4 * nside)


@pytest.mark.parametrize("nside", [2, 8, 32])
def test_north_south_mirror(nside):
    rt = ring_table(nside)
    nr = len(rt["n"])
    for r in range(nr):
        s = nr - 1 - r
        assert rt["z"][r] == pytest.approx(-rt["z"][s], abs=1e-15)
        assert rt["n"][r] == rt["n"][s]
        assert rt["phi0"][r] == pytest.approx(rt["phi0"][s], abs=1e-15)


@pytest.mark.parametrize("nside", [2, 4, 16])
def test_point_set_maps_onto_itself(nside):
    """lambda -> lambda + pi/2 and lambda -> -lambda permute every ring."""
    rt = ring_table(nside)
    for r in range(len(rt["n"])):
        n = int(rt["n"][r])
        lam = rt["phi0"][r] + 2 * np.pi * np.arange(n) / n
        key = lambda v: np.sort(np.round(np.mod(v, 2 * np.pi) / (2 * np.pi) * 4 * n) % (4 * n))
        assert np.array_equal(key(lam), key(lam + np.pi / 2))
        assert np.array_equal(key(lam), key(-lam))


def test_equatorial_shift_rule_matches_ring_parity():
    """Unshifted belt rings (first point at lambda = 0) are the odd-numbered ones."""
    nside = 8
    rt = ring_table(nside)
    for r in range(nside, 3 * nside + 1):
        expect = 0.0 if r % 2 == 1 else np.pi / (4 * nside)
        assert rt["phi0"][r - 1] == pytest.approx(expect)


@pytest.mark.parametrize("n", [1, 5, 64, 513])
def test_gauss_legendre_against_scipy(n):
    x, w = gauss_legendre(n)
    xs, ws = sp.roots_legendre(n)
    assert np.max(np.abs(x - xs)) < 1e-14
    # scipy's own weights carry ~1e-9 relative error near the ends at n = 513
    assert np.max(np.abs(w - ws) / ws) < 1e-8
    # exact for x^k, k <= 2n-1, and for the orthonormal Legendre polynomials
    for k in (0, 1, 2 * n - 2, 2 * n - 1):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert np.sum(w * x ** k) == pytest.approx(exact, abs=1e-13)
    P = plm_orthonormal(n - 1, 0, x)
    G = (P * w[None, :]) @ P.T
    assert np.max(np.abs(G - np.eye(n))) < 1e-13


@pytest.mark.parametrize("l,m", [(0, 0), (1, 0), (1, 1), (5, 3), (30, 17), (60, 60), (120, 7)])
def test_ylm_matches_scipy(l, m):
    th = np.linspace(0.01, np.pi - 0.01, 17)
    lam = np.linspace(0.0, 6.0, 17)
    for mm in (m, -m):
        a = ylm(l, mm, th, lam)
        b = sp.sph_harm_y(l, mm, th, lam)
        assert np.max(np.abs(a - b)) < 1e-13 * max(1.0, np.sqrt(l))


def test_orthonormality_low_and_high_order():
    lmax = 1500
    x, w = gauss_legendre(lmax + 1)
    for m in (0, 1, 2, 600, 1400):
        P = plm_orthonormal(lmax, m, x)
        G = (P * w[None, :]) @ P.T
        assert np.max(np.abs(G - np.eye(lmax - m + 1))) < 1e-11, m


def test_exponent_tracking_keeps_values_that_start_below_double_range():
    """(1 - x^2)^{m/2} underflows at m = 700, x = cos(0.25); Pt_l^m is O(1) at l = 4000."""
    m, l, theta = 700, 4000, 0.25
    x = np.array([np.cos(theta)])
    assert np.sin(theta) ** m == 0.0          # the naive seed underflows
    v = plm_orthonormal(l, m, x)[l - m, 0]
    assert np.isfinite(v) and abs(v) > 1e-3
    # unit norm of that function under quadrature that resolves it
    xq, wq = gauss_legendre(l + 1)
    Pq = plm_orthonormal(l, m, xq)[l - m]
    assert np.sum(wq * Pq * Pq) == pytest.approx(1.0, abs=1e-10)


def test_rows_generator_matches_per_order_recurrence():
    x = np.linspace(-0.999, 0.999, 9)
    for l, P in plm_rows(64, x):
        if l in (0, 1, 2, 33, 64):
            for m in range(l + 1):
                np.testing.assert_allclose(P[m], plm_orthonormal(l, m, x)[l - m], rtol=1e-12, atol=1e-14)
