"""O_plain: HP2SPH (Algorithm 1 of the paper) step by step, FP64 (oracle).

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

Band.  Step 2 truncates the colatitude least-squares fit to 4 Nside + 1
Fourier modes (Sec. 3.2.2), i.e. j = -p..p with p = 2 Nside, and Step 3 then
works with p = 2 Nside in both directions (Sec. 3.3; the source prints
"p = N_side/2", which contradicts the 4 Nside + 1 truncation and the index
ranges next to it, so p = 2 Nside is read).  The output holds l <= p; a
requested lmax < p truncates that result.

The steps, with the readings taken where the paper is silent:

 Step 1 (Sec. 3.1, eqs. upsamp, trig_expansion, interp_cond).  On each ring
   with n points and first longitude phi0 the trigonometric interpolant is
   f_r(lambda) = sum_k c_k e^{i k lambda}; the shifted coefficients
   ct_k = (1/n) sum_q f_q e^{-2 pi i k q / n} come from an FFT and
   c_k = ct_k e^{-i k phi0}.  The Nyquist term (|k| = n/2) is split
   symmetrically so that the interpolant is real:
   c_{+-n/2} = (alpha/2) e^{-+ i (n/2) phi0}, alpha = (1/n) sum_q f_q (-1)^q.
   The interpolant is evaluated on lambda_t = t pi / (2 Nside),
   t = 0 .. 4 Nside - 1, giving the (4 Nside - 1) x 4 Nside tensor grid.
 Poles (Sec. 3.2.1, last paragraph before the Remark).  A quadratic
   least-squares fit (polynomials of degree <= 2 in x, y, z restricted to the
   sphere, equal weights) to the pixels of the three rings nearest each pole,
   evaluated at the pole.
 Step 2(i) (eq. DFS).  The 8 Nside x 4 Nside doubled grid: rows
   theta = 0 (north pole value), theta_1 .. theta_{4Nside-1}, pi (south pole
   value), then 2 pi - theta_r holding f(lambda + pi, theta_r).
 Step 2(ii) (eqs. nufft2, normal_eq; Sec. 3.2.2).  Per longitude column,
   the least-squares fit by sum_{j=-p}^{p} X_j e^{i j theta} over the 8 Nside
   rows, solved exactly (dense QR; this is the limit the paper's CG on the
   normal equations converges to).
 Step 2(iii).  DFT in longitude: C_{jk} = (1/4Nside) sum_t Xhat_j(lambda_t)
   e^{-i k lambda_t}, k = -p .. p-1.
 Step 3 (Sec. 3.3).  X_{j,k} = C_{j,k} for |k| < p and X_{j,+-p} = C_{j,-p}/2;
   then for even k the cosine series G_k(theta) = X_0 + sum_{j>=1}
   (X_{j,k} + X_{-j,k}) cos(j theta), for odd k the sine series
   G_k(theta) = sum_{j>=1} i (X_{j,k} - X_{-j,k}) sin(j theta).  (The printed
   algebra has stray conjugates and a 1/i; these are the forms that
   reproduce sum_j X_j e^{i j theta} on the sphere.)  The FSHT result is the
   L2 projection onto the spherical harmonics of degree <= p:
   a_l^m = s_m sqrt(2 pi) int_{-1}^{1} G_m(arccos x) Pt_l^{|m|}(x) dx, with
   s_m = 1 for m >= 0 and (-1)^m for m < 0 (from Y_l^{-m} = (-1)^m conj(Y_l^m)),
   evaluated by Gauss-Legendre quadrature on p + 2 nodes, which is exact
   because the integrand is a polynomial of degree <= 2p (for odd m both
   factors carry one sqrt(1 - x^2)).

Parity: pinned (see tests/test_oracle_*.py): constant map, real-map
symmetry, the exact equivariances of the point set, exact recovery of
Y_l^{+-1} and Y_0^0, Y_1^0, Y_2^0, consistency of the colatitude fit on
trigonometric polynomials, the unweighted normal equations of that fit on
data it cannot fit exactly (equal weights on all doubled-grid rows), the
re-expansion of X over k = -p..p onto the fitted columns (the half split of
the k = +-p columns), and agreement of the spatial route (this module's
analyze_full) with the Fourier-space route of the Remark in Sec. 3.2.1
(analyze_columns).
"""

import numpy as np
import scipy.linalg

from .geometry import ring_table, pixel_xyz
from .legendre import gauss_legendre, plm_orthonormal, plm_rows


# --------------------------------------------------------------------------
# Step 1: per-ring trigonometric interpolation
# --------------------------------------------------------------------------

def ring_coefficients(f, nside):
    """c_k, k = -n/2 .. n/2, of the real trigonometric interpolant of each ring.

    Returns a list (one entry per ring, north to south) of complex arrays of
    length n + 1 whose index i holds k = i - n/2.
    """
    rt = ring_table(nside)
    out = []
    for r in range(len(rt["n"])):
        n = int(rt["n"][r])
        x = np.asarray(f[rt["start"][r]:rt["start"][r] + n], dtype=np.float64)
        ct = np.fft.fft(x) / n                            # ct_k, k = 0 .. n-1 (mod n)
        k = np.arange(-n // 2, n // 2 + 1)
        c = ct[k % n] * np.exp(-1j * k * rt["phi0"][r])
        alpha = np.sum(x * (-1.0) ** np.arange(n)) / n
        half = n // 2
        c[0] = 0.5 * alpha * np.exp(+1j * half * rt["phi0"][r])    # k = -n/2
        c[-1] = 0.5 * alpha * np.exp(-1j * half * rt["phi0"][r])   # k = +n/2
        out.append(c)
    return out


def upsampled_grid(f, nside):
    """The (4 Nside - 1) x 4 Nside tensor grid of Step 1 (eq. upsamp)."""
    coefs = ring_coefficients(f, nside)
    nl = 4 * nside
    grid = np.empty((len(coefs), nl))
    for r, c in enumerate(coefs):
        n = len(c) - 1
        k = np.arange(-n // 2, n // 2 + 1)
        spec = np.zeros(nl, dtype=np.complex128)
        np.add.at(spec, k % nl, c)                        # sum_k c_k e^{i k lambda_t}
        vals = np.fft.ifft(spec) * nl
        grid[r] = vals.real
    return grid


# --------------------------------------------------------------------------
# Pole values
# --------------------------------------------------------------------------

def _quadratic_basis(xyz, t):
    """Polynomials of degree <= 2 in x, y, z restricted to the sphere.

    With t = 1 - z * pole_z (the distance in z from the pole) the
    nine-dimensional space is spanned by {1, t, t^2, x, y, x t, y t,
    x^2 - y^2, x y} (on the sphere x^2 + y^2 = 2t - t^2 and z = pole_z (1 - t)),
    a basis free of the near-collinear columns that monomials in z have close
    to the pole.  Every function except the constant vanishes at the pole.
    t is passed in from the exact ring geometry (1 - |z| of the cap rings).
    """
    x, y = xyz[:, 0], xyz[:, 1]
    return np.stack([np.ones_like(x), t, t * t, x, y, x * t, y * t, x * x - y * y, x * y], axis=1)


def pole_values(f, nside):
    """(f_N, f_S): quadratic least-squares fit to the three rings nearest each pole.

    Equal weights on the pixels of the three rings (the paper names no
    weighting); the value of the fitted polynomial at the pole is its
    constant coefficient in the basis of _quadratic_basis.
    """
    rt = ring_table(nside)
    xyz = pixel_xyz(nside)
    f = np.asarray(f, dtype=np.float64)
    nr = len(rt["n"])
    res = []
    for rings in ((0, 1, 2), (nr - 1, nr - 2, nr - 3)):
        idx = np.concatenate([np.arange(rt["start"][r], rt["start"][r] + rt["n"][r]) for r in rings])
        t = np.concatenate([np.full(rt["n"][r], rt["one_minus_abs_z"][r]) for r in rings])
        M = _quadratic_basis(xyz[idx], t)
        scale = np.max(np.abs(M), axis=0)
        coef, *_ = np.linalg.lstsq(M / scale[None, :], f[idx], rcond=None)
        res.append(float(coef[0] / scale[0]))
    return res[0], res[1]


# --------------------------------------------------------------------------
# Step 2: DFS + colatitude least squares + longitude DFT
# --------------------------------------------------------------------------

def dfs_thetas(nside):
    """Colatitudes of the 8 Nside rows of the doubled grid (eq. DFS)."""
    th = ring_table(nside)["theta"]
    return np.concatenate([[0.0], th, [np.pi], 2.0 * np.pi - th[::-1]])


def dfs_grid(f, nside):
    """The 8 Nside x 4 Nside doubled grid of Step 2(i)."""
    up = upsampled_grid(f, nside)
    fn, fs = pole_values(f, nside)
    nl = 4 * nside
    half = 2 * nside                                       # lambda + pi = index + 2 Nside
    rows = [np.full(nl, fn)]
    rows += [up[r] for r in range(up.shape[0])]
    rows += [np.full(nl, fs)]
    rows += [np.roll(up[r], -half) for r in range(up.shape[0] - 1, -1, -1)]
    return np.array(rows)


class _ColatitudeLSQ:
    """Least squares by e^{i j theta}, j = -p..p, on the doubled-grid rows (QR)."""

    def __init__(self, nside):
        p = 2 * nside
        self.p = p
        th = dfs_thetas(nside)
        j = np.arange(-p, p + 1)
        self.E = np.exp(1j * np.outer(th, j))             # (8 Nside) x (4 Nside + 1)
        self.Q, self.R = scipy.linalg.qr(self.E, mode="economic")

    def solve(self, d):
        return scipy.linalg.solve_triangular(self.R, self.Q.conj().T @ d)


_LSQ_CACHE = {}


def _lsq(nside):
    if nside not in _LSQ_CACHE:
        _LSQ_CACHE.clear()
        _LSQ_CACHE[nside] = _ColatitudeLSQ(nside)
    return _LSQ_CACHE[nside]


def bivariate_coefficients(f, nside):
    """X_{j,k}, j, k = -p..p (array index [j + p, k + p]), Steps 2 and 3 set-up."""
    p = 2 * nside
    grid = dfs_grid(f, nside)
    xhat = _lsq(nside).solve(grid.astype(np.complex128))  # (4 Nside + 1) x (4 Nside)
    nl = 4 * nside
    C = np.fft.fft(xhat, axis=1) / nl                      # column index = k mod 4 Nside
    X = np.zeros((2 * p + 1, 2 * p + 1), dtype=np.complex128)
    for k in range(-p + 1, p):
        X[:, k + p] = C[:, k % nl]
    X[:, 0] = 0.5 * C[:, (-p) % nl]
    X[:, 2 * p] = 0.5 * C[:, (-p) % nl]
    return X


def trig_series(X, p):
    """Cosine and sine coefficients per longitude mode k (Sec. 3.3, corrected).

    Returns (A, B): A[j, k + p], j = 0..p, the cosine series of
    sum_j X_{j,k} e^{i j theta}; B[j, k + p], j = 1..p (row 0 unused), its sine
    series.  For a function on the sphere the odd-k cosine and even-k sine
    parts vanish.
    """
    A = np.zeros((p + 1, 2 * p + 1), dtype=np.complex128)
    B = np.zeros((p + 1, 2 * p + 1), dtype=np.complex128)
    A[0] = X[p]
    for j in range(1, p + 1):
        A[j] = X[p + j] + X[p - j]
        B[j] = 1j * (X[p + j] - X[p - j])
    return A, B


# --------------------------------------------------------------------------
# Step 3: spherical-harmonic coefficients (L2 projection)
# --------------------------------------------------------------------------

def _project(G_at_nodes, ks, nodes, weights, lmax):
    """a[l, i] = sqrt(2 pi) sum_q w_q G_i(x_q) Pt_l^{|k_i|}(x_q) (-1)^{k_i}[k_i<0].

    G_at_nodes[i, q] holds G_{k_i}(arccos x_q).
    """
    ks = np.asarray(ks)
    am = np.abs(ks)
    sign = np.where(ks < 0, (-1.0) ** am, 1.0)
    wg = G_at_nodes * weights[None, :]
    out = np.zeros((lmax + 1, len(ks)), dtype=np.complex128)
    if len(ks) <= 8:
        # few orders: one recurrence per order instead of all orders at once
        for i, k in enumerate(ks):
            a = abs(int(k))
            if a > lmax:
                continue
            P = plm_orthonormal(lmax, a, nodes)           # rows l = |k| .. lmax
            out[a:, i] = np.sqrt(2.0 * np.pi) * sign[i] * (P @ wg[i])
        return out
    for l, P in plm_rows(lmax, nodes):
        sel = am <= l
        if not np.any(sel):
            continue
        rows = P[am[sel]]                                  # Pt_l^{|k|}(x_q)
        out[l, sel] = np.sqrt(2.0 * np.pi) * sign[sel] * np.sum(wg[sel] * rows, axis=1)
    return out


def _series_at_nodes(A, B, ks, p, theta_nodes):
    j = np.arange(p + 1)
    cosm = np.cos(np.outer(theta_nodes, j))                # (nq, p+1)
    sinm = np.sin(np.outer(theta_nodes, j))
    G = np.empty((len(ks), len(theta_nodes)), dtype=np.complex128)
    for i, k in enumerate(ks):
        if k % 2 == 0:
            G[i] = cosm @ A[:, k + p]
        else:
            G[i] = sinm @ B[:, k + p]
    return G


def analyze_full(f, nside, lmax=None, return_intermediates=False):
    """All a_l^m, -l <= m <= l <= lmax, by the spatial route of Algorithm 1.

    Returns an array a[l, m + lmax] (zero where |m| > l).
    """
    p = 2 * nside
    lmax = p if lmax is None else int(lmax)
    if not 0 <= lmax <= p:
        raise ValueError("0 <= lmax <= 2 nside")
    X = bivariate_coefficients(f, nside)
    A, B = trig_series(X, p)
    nodes, weights = gauss_legendre(p + 2)
    ks = np.arange(-lmax, lmax + 1)
    G = _series_at_nodes(A, B, ks, p, np.arccos(nodes))
    a = _project(G, ks, nodes, weights, lmax)
    if return_intermediates:
        return a, {"X": X, "A": A, "B": B}
    return a


def pack_nonnegative(a_full, lmax):
    """Packed m-major layout for m >= 0: index m (2 lmax + 1 - m) / 2 + l."""
    out = np.zeros((lmax + 1) * (lmax + 2) // 2, dtype=np.complex128)
    for m in range(lmax + 1):
        base = m * (2 * lmax + 1 - m) // 2
        out[base + m:base + lmax + 1] = a_full[m:lmax + 1, m + lmax]
    return out


def analyze(f, nside, lmax=None):
    """a_l^m for 0 <= m <= l <= lmax, packed m-major (see pack_nonnegative)."""
    p = 2 * nside
    lmax = p if lmax is None else int(lmax)
    if not 0 <= lmax <= p:
        raise ValueError("0 <= lmax <= 2 nside")
    X = bivariate_coefficients(f, nside)
    A, B = trig_series(X, p)
    nodes, weights = gauss_legendre(p + 2)
    ks = np.arange(0, lmax + 1)
    G = _series_at_nodes(A, B, ks, p, np.arccos(nodes))
    a = _project(G, ks, nodes, weights, lmax)             # a[l, m]
    out = np.zeros((lmax + 1) * (lmax + 2) // 2, dtype=np.complex128)
    for m in range(lmax + 1):
        base = m * (2 * lmax + 1 - m) // 2
        out[base + m:base + lmax + 1] = a[m:, m]
    return out


def analyze_columns(f, nside, ms, lmax=None):
    """a_l^m, l = |m| .. lmax, for the listed orders only (Fourier-space route).

    Uses the Remark of Sec. 3.2.1: the doubled grid is formed in longitude
    Fourier space -- the column for mode k holds the rings' mode-k
    coefficients of the upsampled rows (north to south), then the same
    coefficients of the rings south to north times (-1)^k, with the pole
    values in the k = 0 column only -- so one order needs only its own column.
    Returns {m: complex array of a_l^m for l = |m| .. lmax}.
    """
    p = 2 * nside
    lmax = p if lmax is None else int(lmax)
    coefs = ring_coefficients(f, nside)
    fn, fs = pole_values(f, nside)
    nl = 4 * nside
    lsq = _lsq(nside)
    nodes, weights = gauss_legendre(p + 2)
    res = {}
    for m in ms:
        # upsampled-row coefficient at mode k (for k = +-p, the grid Nyquist mode -p)
        kk = -p if abs(m) == p else m
        col_r = np.empty(len(coefs), dtype=np.complex128)
        for r, c in enumerate(coefs):
            n = len(c) - 1
            k = np.arange(-n // 2, n // 2 + 1)
            col_r[r] = np.sum(c[(k - kk) % nl == 0])
        sgn = (-1.0) ** kk
        d = np.concatenate([[fn if kk == 0 else 0.0], col_r, [fs if kk == 0 else 0.0], sgn * col_r[::-1]])
        x = lsq.solve(d)
        if abs(m) == p:
            x = 0.5 * x
        X = np.zeros((2 * p + 1, 2 * p + 1), dtype=np.complex128)
        X[:, m + p] = x
        A, B = trig_series(X, p)
        G = _series_at_nodes(A, B, [m], p, np.arccos(nodes))
        a = _project(G, [m], nodes, weights, lmax)
        res[m] = a[abs(m):, 0]
    return res
