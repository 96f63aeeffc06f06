"""Pins of the equal-weight analysis and its Jacobi iteration (oracle/healpix.py).

The oracle evaluates eq. (healsph) through per-ring longitude sums and
Legendre sums; these tests hold it against routes that share none of that:
the dense synthesis matrix S of all Y_l^m at the pixel centres (dense.py,
pinned by the printed Table 1), closed forms, and the least-squares solution.
"""

import numpy as np
import pytest

import oracle as O
from oracle.dense import synthesis_matrix
from oracle.healpix import analyze_equal_weight, analyze_jacobi
import workloads as W


def _pack_from_dense(v, lmax):
    """Column order (l, m = -l..l) of synthesis_matrix -> packed m >= 0."""
    out = np.zeros((lmax + 1) * (lmax + 2) // 2, dtype=np.complex128)
    i = 0
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            if m >= 0:
                out[O.alm_index(l, m, lmax)] = v[i]
            i += 1
    return out


def _unpack_to_dense(a, lmax):
    """Packed m >= 0 of a real map -> all m, a_l^{-m} = (-1)^m conj(a_l^m)."""
    out = []
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            v = a[O.alm_index(l, abs(m), lmax)]
            out.append(v if m >= 0 else (-1) ** m * np.conj(v))
    return np.array(out)


def _full_norm(a, lmax):
    """Euclidean norm over all m of the real-map coefficient vector."""
    return np.linalg.norm(_unpack_to_dense(a, lmax))


@pytest.mark.parametrize("nside,lmax", [(2, 4), (2, 5), (4, 8), (4, 11)])
def test_equal_weight_matches_dense_route(nside, lmax):
    """(4 pi / N) S^H f from the dense matrix, for lmax below and above the
    Nyquist mode of the polar rings (lmax = 3 Nside - 1 is the HEALPix default)."""
    f = W.random_map(O.npix(nside), W.rng_for(30, nside * 100 + lmax))
    S = synthesis_matrix(nside, lmax)
    N = S.shape[0]
    ref = _pack_from_dense((4.0 * np.pi / N) * (S.conj().T @ f), lmax)
    got = analyze_equal_weight(f, nside, lmax)
    assert np.max(np.abs(got - ref)) < 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("nside,lmax,niter", [(2, 4, 3), (4, 8, 3), (4, 11, 2)])
def test_jacobi_matches_dense_iteration(nside, lmax, niter):
    """eq. (uzawa) run with the dense matrices A = (4 pi / N) S^H and S."""
    f = W.random_map(O.npix(nside), W.rng_for(31, nside * 100 + lmax))
    S = synthesis_matrix(nside, lmax)
    N = S.shape[0]
    A = (4.0 * np.pi / N) * S.conj().T
    a = A @ f
    for _ in range(niter):
        a = a + A @ (f - S @ a)
    ref = _pack_from_dense(a, lmax)
    got = analyze_jacobi(f, nside, lmax, niter)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


def test_constant_map():
    """a_0^0 = sqrt(4 pi) c exactly; every ring is invariant under a quarter
    turn in longitude, so orders not divisible by 4 vanish."""
    nside, lmax, c = 4, 11, 1.75
    a = analyze_equal_weight(np.full(O.npix(nside), c), nside, lmax)
    assert abs(a[O.alm_index(0, 0, lmax)] - np.sqrt(4.0 * np.pi) * c) < 1e-14
    for m in range(lmax + 1):
        if m % 4:
            for l in range(m, lmax + 1):
                assert abs(a[O.alm_index(l, m, lmax)]) < 1e-14


@pytest.mark.parametrize("nside", [2, 4, 8])
def test_jacobi_error_contracts_by_the_spectral_radius(nside):
    """On band-limited input f = S a (lmax = 2 Nside, S of full column rank),
    the error after k iterations is (I - (4 pi / N) S^* S)^(k+1) a, so its norm
    is at most rho^(k+1) |a| with rho the spectral radius (its lambda_max - 1
    part is Table 1's printed value)."""
    lmax = 2 * nside
    a_true = W.draw_alm(np.ones(lmax + 1), lmax, W.rng_for(32, nside))
    f = O.synthesize(a_true, nside, lmax)
    up, down = O.richardson_radius_readings(nside, lmax)
    rho = max(up, down)
    norm = _full_norm(a_true, lmax)
    prev = None
    for k in range(4):
        e = _full_norm(analyze_jacobi(f, nside, lmax, k) - a_true, lmax)
        assert e <= rho ** (k + 1) * norm * (1.0 + 1e-9) + 1e-13 * norm
        if prev is not None:
            assert e < prev
        prev = e


def test_jacobi_fixed_point_is_least_squares():
    """Iterated to convergence, eq. (richardson) gives the least-squares
    solution of S a = f (O_dense), also for input that is not band-limited."""
    nside, lmax = 2, 4
    f = W.random_map(O.npix(nside), W.rng_for(33, 0))
    dense = O.analyze_dense(f, nside, lmax)
    ref = np.zeros((lmax + 1) * (lmax + 2) // 2, dtype=np.complex128)
    for l in range(lmax + 1):
        for m in range(l + 1):
            ref[O.alm_index(l, m, lmax)] = dense[l, m + lmax]
    got = analyze_jacobi(f, nside, lmax, 60)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))
    # a single equal-weight pass is visibly off (the quadrature is not exact)
    assert np.max(np.abs(analyze_equal_weight(f, nside, lmax) - ref)) > 1e-3 * np.max(np.abs(ref))


def test_per_order_route_matches_full_analysis():
    """equal_weight_columns (order-m Legendre functions evaluated directly)
    equals analyze_equal_weight (the l-recurrence of all orders)."""
    nside, lmax = 8, 16
    f = W.random_map(O.npix(nside), W.rng_for(34, 0))
    full = analyze_equal_weight(f, nside, lmax)
    cols = O.equal_weight_columns(f, nside, [0, 1, 5, 15, 16], lmax)
    for m, v in cols.items():
        ref = np.array([full[O.alm_index(l, m, lmax)] for l in range(m, lmax + 1)])
        assert np.max(np.abs(v - ref)) < 1e-14 * np.max(np.abs(full))
