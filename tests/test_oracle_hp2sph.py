"""Pins of O_plain (HP2SPH oracle) against what the paper and the mathematics fix."""

import os

import numpy as np
import pytest

import oracle as O
from oracle import hp2sph as H
from oracle.geometry import ring_table, pixel_angles, pixel_xyz
from oracle.legendre import ylm

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rand_map(nside, seed=0):
    return np.random.default_rng(seed).standard_normal(O.npix(nside))


def _expected_single(l, m, lmax, part="re"):
    """Coefficients of Re(Y_l^m) (or Im) for m >= 0 as a[l, m + lmax]."""
    a = np.zeros((lmax + 1, 2 * lmax + 1), dtype=np.complex128)
    if m == 0:
        a[l, lmax] = 1.0 if part == "re" else 0.0
    elif part == "re":       # Re Y = (Y_l^m + (-1)^m Y_l^{-m}) / 2
        a[l, lmax + m] = 0.5
        a[l, lmax - m] = 0.5 * (-1) ** m
    else:                    # Im Y = (Y_l^m - (-1)^m Y_l^{-m}) / (2i)
        a[l, lmax + m] = -0.5j
        a[l, lmax - m] = 0.5j * (-1) ** m
    return a


@pytest.mark.parametrize("nside", [2, 4, 16])
def test_constant_map(nside):
    c = 2.5
    a = O.analyze_full(np.full(O.npix(nside), c), nside)
    p = 2 * nside
    assert a[0, p] == pytest.approx(np.sqrt(4 * np.pi) * c, rel=1e-14)
    rest = a.copy()
    rest[0, p] = 0
    assert np.max(np.abs(rest)) < 1e-13


@pytest.mark.parametrize("nside", [4, 8])
def test_real_map_symmetry(nside):
    p = 2 * nside
    a = O.analyze_full(_rand_map(nside, 1), nside)
    ms = np.arange(-p, p + 1)
    assert np.max(np.abs(a[:, ::-1] * ((-1.0) ** ms)[None, :] - np.conj(a))) < 1e-14
    assert np.max(np.abs(a[:, p].imag)) < 1e-15


@pytest.mark.parametrize("nside", [4, 8])
def test_exact_recovery_where_the_method_is_exact(nside):
    """Y_l^{+-1} (every l <= p), Y_0^0, Y_1^0, Y_2^0 come back to rounding."""
    p = 2 * nside
    th, lam = pixel_angles(nside)
    cases = [(l, 1, part) for l in (1, 2, p // 2 + 1, p) for part in ("re", "im")]
    cases += [(0, 0, "re"), (1, 0, "re"), (2, 0, "re")]
    for l, m, part in cases:
        y = ylm(l, m, th, lam)
        f = y.real if part == "re" else y.imag
        a = O.analyze_full(f, nside)
        assert np.max(np.abs(a - _expected_single(l, m, p, part))) < 1e-12, (l, m, part)


def test_method_is_not_exact_for_higher_orders_or_zonal_degree_3():
    """Polar rings alias |m| >= 2j, and the pole rule is exact only for l <= 2."""
    nside = 8
    p = 2 * nside
    th, lam = pixel_angles(nside)
    for l, m in ((3, 0), (2, 2), (4, 2), (10, 7)):
        f = ylm(l, m, th, lam).real
        a = O.analyze_full(f, nside)
        assert np.max(np.abs(a - _expected_single(l, m, p))) > 1e-8, (l, m)


@pytest.mark.parametrize("nside", [4, 8])
def test_exact_equivariances(nside):
    """Maps of the point set onto itself act exactly on the coefficients."""
    p = 2 * nside
    rt = ring_table(nside)
    f = _rand_map(nside, 2)
    a = O.analyze_full(f, nside)
    ms = np.arange(-p, p + 1)
    ells = np.arange(p + 1)
    # lambda -> lambda + pi/2: f'(lambda) = f(lambda - pi/2), a' = e^{-i m pi/2} a
    g = np.empty_like(f)
    for r in range(len(rt["n"])):
        s, n = rt["start"][r], rt["n"][r]
        g[s:s + n] = np.roll(f[s:s + n], n // 4)
    ag = O.analyze_full(g, nside)
    assert np.max(np.abs(ag - a * np.exp(-1j * ms * np.pi / 2)[None, :])) < 1e-13
    # z -> -z: rings r and 4 Nside - r swap, a' = (-1)^{l+m} a
    g = np.empty_like(f)
    nr = len(rt["n"])
    for r in range(nr):
        s, n = rt["start"][r], rt["n"][r]
        t = rt["start"][nr - 1 - r]
        g[s:s + n] = f[t:t + n]
    ag = O.analyze_full(g, nside)
    par = (-1.0) ** (ells[:, None] + ms[None, :])
    assert np.max(np.abs(ag - par * a)) < 1e-13
    # lambda -> -lambda: a' = conj(a)
    g = np.empty_like(f)
    for r in range(nr):
        s, n = rt["start"][r], rt["n"][r]
        q = np.arange(n)
        src = (-q) % n if rt["phi0"][r] == 0.0 else (-q - 1) % n
        g[s:s + n] = f[s + src]
    ag = O.analyze_full(g, nside)
    assert np.max(np.abs(ag - np.conj(a))) < 1e-13


@pytest.mark.parametrize("nside", [2, 4, 8])
def test_spatial_route_equals_fourier_space_route(nside):
    """Algorithm 1 literally (grid, DFS, fit, DFT) == the Remark's Fourier-space DFS."""
    p = 2 * nside
    f = _rand_map(nside, 3)
    a = O.analyze_full(f, nside)
    cols = O.analyze_columns(f, nside, list(range(-p, p + 1)))
    for m, v in cols.items():
        assert np.max(np.abs(v - a[abs(m):, m + p])) < 1e-14, m


@pytest.mark.parametrize("nside", [2, 8])
def test_colatitude_fit_recovers_trig_polynomials(nside):
    p = 2 * nside
    rng = np.random.default_rng(4)
    X = rng.standard_normal(2 * p + 1) + 1j * rng.standard_normal(2 * p + 1)
    th = H.dfs_thetas(nside)
    d = np.exp(1j * np.outer(th, np.arange(-p, p + 1))) @ X
    assert np.max(np.abs(H._lsq(nside).solve(d) - X)) < 1e-12


@pytest.mark.parametrize("nside", [2, 4, 8])
def test_bivariate_coefficients_reexpand_to_the_fitted_columns(nside):
    """Sec. 3.3: summed over k = -p..p against e^{i k lambda_t} on the longitude
    nodes lambda_t = t pi / (2 Nside), the X array gives back the colatitude
    series fitted to every column of the doubled grid.  On the nodes
    e^{i p lambda_t} = e^{-i p lambda_t}, so the two k = +-p columns must add up
    to the single grid Nyquist coefficient C_{-p}: this fixes the half weights
    of the split (the real-map symmetry, pinned above on all orders, fixes that
    the two halves are equal)."""
    p = 2 * nside
    f = _rand_map(nside, 11)
    X = H.bivariate_coefficients(f, nside)
    # the fitted colatitude series of every longitude column, straight from the
    # least-squares fit of the doubled grid
    xhat = H._lsq(nside).solve(H.dfs_grid(f, nside).astype(np.complex128))
    lam = np.arange(4 * nside) * np.pi / (2 * nside)
    k = np.arange(-p, p + 1)
    back = X @ np.exp(1j * np.outer(k, lam))
    assert np.max(np.abs(back - xhat)) < 1e-13 * np.max(np.abs(xhat))
    # the input has Nyquist content (unshifted belt rings), so the split matters
    assert np.max(np.abs(X[:, 0])) > 1e-3 * np.max(np.abs(X))


def _dfs_colatitudes(nside):
    """The 8 Nside doubled-grid colatitudes built here from eq. (healpts):
    north pole, rings 1 .. 4 Nside - 1, south pole, then 2 pi - theta_r."""
    ns = float(nside)
    th = []
    for r in range(1, 4 * nside):
        j = min(r, 4 * nside - r)
        if j < nside:
            z = 1.0 - j * j / (3.0 * ns * ns)
            t = 2.0 * np.arcsin(j / (np.sqrt(6.0) * ns))    # 1 - cos t = j^2 / (3 Nside^2)
            th.append(t if r < nside else np.pi - t)
            assert abs(np.cos(th[-1]) - (z if r < nside else -z)) < 1e-14
        else:
            th.append(np.arccos(2.0 * (2 * nside - r) / (3.0 * ns)))
    th = np.array(th)
    return np.concatenate([[0.0], th, [np.pi], 2.0 * np.pi - th[::-1]])


@pytest.mark.parametrize("nside", [2, 4, 8])
def test_colatitude_fit_solves_the_unweighted_normal_equations(nside):
    """Sec. 3.2.2, eqs. normal_eq and equigrid: the fit minimises the plain sum
    of squares over all 8 Nside doubled-grid rows (pole rows weighted like any
    other).  On data that no trigonometric polynomial of degree p fits, the
    residual d - E x must be orthogonal to every column of E_{s,j} =
    e^{i j theta_s}, j = -p..p, i.e. E^H E x = E^H d.  A weighted fit (say the
    pole rows counted three times) leaves a residual that is not."""
    p = 2 * nside
    theta = _dfs_colatitudes(nside)
    assert np.allclose(theta, H.dfs_thetas(nside), rtol=0, atol=1e-14)
    E = np.exp(1j * np.outer(theta, np.arange(-p, p + 1)))
    rng = np.random.default_rng(12)
    d = rng.standard_normal(8 * nside) + 1j * rng.standard_normal(8 * nside)
    x = H._lsq(nside).solve(d)
    res = d - E @ x
    assert np.linalg.norm(res) > 0.1 * np.linalg.norm(d)          # not an exact fit
    assert np.max(np.abs(E.conj().T @ res)) < 1e-12 * np.max(np.abs(E.conj().T @ d))
    # the normal matrix is the Toeplitz matrix of the sums of e^{i q theta_s}
    q = np.arange(-2 * p, 2 * p + 1)
    t = np.exp(1j * np.outer(q, theta)).sum(axis=1)
    jj = np.arange(-p, p + 1)
    assert np.max(np.abs(E.conj().T @ E - t[(jj[None, :] - jj[:, None]) + 2 * p])) < 1e-11


def test_doubled_grid_gives_sphere_parity():
    """On the doubled grid even-k columns are cosine series and odd-k sine series."""
    nside = 8
    p = 2 * nside
    X = H.bivariate_coefficients(_rand_map(nside, 5), nside)
    A, B = H.trig_series(X, p)
    ks = np.arange(-p, p + 1)
    assert np.max(np.abs(A[:, ks % 2 == 1])) < 1e-14
    assert np.max(np.abs(B[1:, ks % 2 == 0])) < 1e-14
    assert np.max(np.abs(A[:, ks % 2 == 0])) > 1e-2


@pytest.mark.parametrize("nside", [2, 4, 16])
def test_ring_interpolant_is_real_and_interpolates(nside):
    f = _rand_map(nside, 6)
    rt = ring_table(nside)
    coefs = H.ring_coefficients(f, nside)
    for r, c in enumerate(coefs):
        n = len(c) - 1
        k = np.arange(-n // 2, n // 2 + 1)
        lam = rt["phi0"][r] + 2 * np.pi * np.arange(n) / n
        vals = np.exp(1j * np.outer(lam, k)) @ c
        assert np.max(np.abs(vals - f[rt["start"][r]:rt["start"][r] + n])) < 1e-13
        off = np.linspace(0, 2 * np.pi, 11)
        assert np.max(np.abs((np.exp(1j * np.outer(off, k)) @ c).imag)) < 1e-13


@pytest.mark.parametrize("nside", [2, 4, 32])
def test_pole_values(nside):
    """Exact for harmonics of degree <= 2; equal to quadratic extrapolation of ring means."""
    th, lam = pixel_angles(nside)
    for l in range(3):
        for m in range(l + 1):
            f = ylm(l, m, th, lam).real
            fn, fs = H.pole_values(f, nside)
            assert fn == pytest.approx(ylm(l, m, np.array([0.0]), np.array([0.0])).real[0], abs=1e-13)
            assert fs == pytest.approx(ylm(l, m, np.array([np.pi]), np.array([0.0])).real[0], abs=1e-13)
    f = _rand_map(nside, 7)
    rt = ring_table(nside)
    fn, fs = H.pole_values(f, nside)
    nr = len(rt["n"])
    for rings, pole, val in (((0, 1, 2), 1.0, fn), ((nr - 1, nr - 2, nr - 3), -1.0, fs)):
        zs = np.array([rt["z"][r] for r in rings])
        mu = np.array([f[rt["start"][r]:rt["start"][r] + rt["n"][r]].mean() for r in rings])
        lag = sum(mu[i] * np.prod([(pole - zs[j]) / (zs[i] - zs[j]) for j in range(3) if j != i]) for i in range(3))
        assert val == pytest.approx(lag, abs=1e-12)
    if nside >= 4:   # polar rings: weights (3/2, -3/5, 1/10)
        mu = np.array([f[rt["start"][r]:rt["start"][r] + rt["n"][r]].mean() for r in (0, 1, 2)])
        assert fn == pytest.approx(1.5 * mu[0] - 0.6 * mu[1] + 0.1 * mu[2], abs=1e-12)


def _potential_spline():
    rows = [l.split() for l in open(os.path.join(GOLD, "potential_spline.txt")) if l.strip() and not l.startswith("#")]
    return [(float(c), float(la), float(t)) for c, la, t in rows]


def _spline_map(nside):
    xyz = pixel_xyz(nside)
    f = np.zeros(len(xyz))
    for c, la, t in _potential_spline():
        xc = np.array([np.cos(la) * np.sin(t), np.sin(la) * np.sin(t), np.cos(t)])
        f += c * np.maximum(2.0 - 2.0 * xyz @ xc, 0.0) ** 1.5
    return f


def _spline_alm(lmax):
    a = np.zeros((lmax + 1, 2 * lmax + 1), dtype=np.complex128)
    for l in range(lmax + 1):
        fac = 18 * np.pi / ((l + 2.5) * (l + 1.5) * (l + 0.5) * (l - 0.5) * (l - 1.5))
        for m in range(-l, l + 1):
            a[l, m + lmax] = fac * sum(c * np.conj(ylm(l, m, np.array([t]), np.array([la]))[0])
                                       for c, la, t in _potential_spline())
    return a


def test_potential_spline_error_falls_with_resolution():
    """Sec. 4.1 trend (figure values are not printed): the max coefficient error
    against the closed form of eq. (alm) falls as t = log2 Nside grows."""
    errs = []
    for nside in (4, 8, 16, 32):
        p = 2 * nside
        a = O.analyze_full(_spline_map(nside), nside)
        exact = _spline_alm(p)
        errs.append(np.max(np.abs(a - exact)))
    assert all(errs[i + 1] < 0.5 * errs[i] for i in range(len(errs) - 1)), errs
