"""Orthonormal associated Legendre functions and spherical harmonics (oracle).

Conventions of Appendix A, eqs. (ssph) and (sphip):

  Y_l^m(lambda, theta) = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) P_l^m(cos theta) e^{i m lambda}

with P_l^m carrying the Condon-Shortley phase (-1)^m, and for negative order
Y_l^{-m} = (-1)^m conj(Y_l^m).  (The appendix prints Y_l^{-m} = (-1)^m Y_l^{|m|};
taken literally that would make Y_l^{m} and Y_l^{-m} parallel, so the usual
conjugate form is used; it is the form under which a real map satisfies
a_l^{-m} = (-1)^m conj(a_l^m).)

Writing Pt_l^m = sqrt((2l+1)/2 (l-m)!/(l+m)!) P_l^m for the functions that are
orthonormal on [-1, 1], Y_l^m = Pt_l^m(cos theta) e^{i m lambda} / sqrt(2 pi).

Pt_l^m is evaluated by the standard three-term recurrence in l,
  Pt_m^m     = (-1)^m sqrt((2m+1)/2 prod_{i<=m} (2i-1)/(2i)) (1-x^2)^{m/2}
  Pt_{m+1}^m = sqrt(2m+3) x Pt_m^m
  Pt_l^m     = sqrt((4l^2-1)/(l^2-m^2)) x Pt_{l-1}^m
               - sqrt((2l+1)((l-1)^2-m^2)/((2l-3)(l^2-m^2))) Pt_{l-2}^m,
carrying a separate power-of-two exponent so that (1-x^2)^{m/2} underflowing
double range near the poles cannot zero a sequence that grows again later.

Parity pinned by: orthonormality under Gauss-Legendre quadrature, agreement
with scipy.special.sph_harm_y / assoc_legendre_p (independent library code),
and Table 1 of the paper (through the dense synthesis matrix).
"""

import numpy as np

_RESCALE_BITS = 256


def _legendre_pair(n, x):
    """(P_{n-1}(x), P_n(x)) by the three-term recurrence (unnormalised)."""
    p0 = np.ones_like(x)
    p1 = x.copy()
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    return p0, p1


def gauss_legendre(n):
    """Nodes and weights of n-point Gauss-Legendre quadrature on [-1, 1].

    Newton iteration on P_n from the classical Chebyshev-like initial guess,
    with P_n and P_n' from the three-term recurrence.  Exact for polynomials
    of degree <= 2n - 1.
    """
    if n < 1:
        raise ValueError("n >= 1")
    i = np.arange(1, n + 1)
    x = np.cos(np.pi * (i - 0.25) / (n + 0.5))
    for _ in range(12):
        p0, p1 = _legendre_pair(n, x)
        dp = n * (x * p1 - p0) / ((x - 1.0) * (x + 1.0))
        dx = p1 / dp
        x = x - dx
        if np.max(np.abs(dx)) < 1e-15:
            break
    # derivative at the converged nodes, for the weights
    p0, p1 = _legendre_pair(n, x)
    dp = n * (x * p1 - p0) / ((x - 1.0) * (x + 1.0))
    w = 2.0 / ((1.0 - x) * (1.0 + x) * dp * dp)
    order = np.argsort(x)
    return x[order], w[order]


def plm_orthonormal(lmax, m, x):
    """Pt_l^m(x) for l = m .. lmax, as an array of shape (lmax - m + 1, len(x)).

    Values whose magnitude falls below the double range are returned as 0.
    """
    x = np.asarray(x, dtype=np.float64)
    m = int(m)
    if m < 0 or lmax < m:
        raise ValueError("need 0 <= m <= lmax")
    out = np.zeros((lmax - m + 1, x.size))
    s = np.sqrt(np.maximum((1.0 - x) * (1.0 + x), 0.0))
    # log2 of |Pt_m^m| = 0.5 log2((2m+1)/2 prod (2i-1)/(2i)) + m log2(s)
    i = np.arange(1, m + 1, dtype=np.float64)
    logc = 0.5 * (np.log2((2 * m + 1) / 2.0) + np.sum(np.log2((2 * i - 1) / (2 * i))))
    nonzero = (s > 0) | (m == 0)
    with np.errstate(divide="ignore"):
        logv = logc + (m * np.log2(s) if m > 0 else 0.0)
    logv = np.where(nonzero, logv, 0.0)
    e = np.floor(logv).astype(np.int64)
    sign = -1.0 if (m % 2) else 1.0
    cur = np.where(nonzero, sign * np.exp2(logv - e), 0.0)    # mantissa, |.| in [1, 2)
    prev = np.zeros_like(cur)
    out[0] = np.ldexp(cur, e)
    for l in range(m + 1, lmax + 1):
        if l == m + 1:
            nxt = np.sqrt(2.0 * m + 3.0) * x * cur
        else:
            a = np.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
            b = np.sqrt((2.0 * l + 1.0) * ((l - 1.0) ** 2 - m * m) / ((2.0 * l - 3.0) * (l * l - m * m)))
            nxt = a * x * cur - b * prev
        prev, cur = cur, nxt
        big = np.abs(cur) > 2.0 ** _RESCALE_BITS
        if np.any(big):
            cur = np.where(big, np.ldexp(cur, -_RESCALE_BITS), cur)
            prev = np.where(big, np.ldexp(prev, -_RESCALE_BITS), prev)
            e = e + np.where(big, _RESCALE_BITS, 0)
        out[l - m] = np.ldexp(cur, e)
    return out


def ylm(l, m, theta, lam):
    """Y_l^m(lambda, theta) for a single (l, m), any sign of m (Appendix A)."""
    theta = np.asarray(theta, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    am = abs(m)
    p = plm_orthonormal(l, am, np.cos(theta).ravel())[l - am].reshape(theta.shape)
    y = p * np.exp(1j * am * lam) / np.sqrt(2.0 * np.pi)
    if m < 0:
        y = (-1) ** am * np.conj(y)
    return y


def plm_rows(lmax, x, check_every=16):
    """Yield (l, P) for l = 0 .. lmax, where P[m, i] = Pt_l^m(x[i]) for m = 0 .. l.

    The same recurrence as plm_orthonormal, run for every order m at once
    (rows are orders), so that sums over l for all m cost one pass.  Each row
    carries its own power-of-two exponent per point.
    """
    x = np.asarray(x, dtype=np.float64)
    nx = x.size
    s = np.sqrt(np.maximum((1.0 - x) * (1.0 + x), 0.0))
    with np.errstate(divide="ignore"):
        log2s = np.log2(s)
    cur = np.zeros((lmax + 1, nx))
    prev = np.zeros((lmax + 1, nx))
    e = np.zeros((lmax + 1, nx), dtype=np.int64)
    logc = 0.0          # 0.5 log2((2m+1)/2 prod_{i<=m} (2i-1)/(2i)) without the (2m+1)/2 part
    for l in range(lmax + 1):
        m = l
        if m > 0:
            logc += np.log2((2.0 * m - 1.0) / (2.0 * m))
        # seed row m = l
        if m == 0:
            logv = np.full(nx, 0.5 * np.log2(0.5))
            ok = np.ones(nx, dtype=bool)
        else:
            ok = s > 0
            logv = np.where(ok, 0.5 * (np.log2((2 * m + 1) / 2.0) + logc) + m * np.where(ok, log2s, 0.0), 0.0)
        em = np.floor(logv).astype(np.int64)
        sign = -1.0 if (m % 2) else 1.0
        seed = np.where(ok, sign * np.exp2(logv - em), 0.0)
        if l >= 1:
            # row m = l-1: Pt_l^{l-1} = sqrt(2l+1) x Pt_{l-1}^{l-1}
            mm = l - 1
            new1 = np.sqrt(2.0 * mm + 3.0) * x * cur[mm]
            prev[mm] = cur[mm]
            cur[mm] = new1
        if l >= 2:
            mr = np.arange(l - 1, dtype=np.float64)[:, None]
            a = np.sqrt((4.0 * l * l - 1.0) / (l * l - mr * mr))
            b = np.sqrt((2.0 * l + 1.0) * ((l - 1.0) ** 2 - mr * mr) / ((2.0 * l - 3.0) * (l * l - mr * mr)))
            new = a * x[None, :] * cur[:l - 1] - b * prev[:l - 1]
            prev[:l - 1] = cur[:l - 1]
            cur[:l - 1] = new
        cur[l] = seed
        prev[l] = 0.0
        e[l] = em
        if l % check_every == 0:
            big = np.abs(cur[:l + 1]) > 2.0 ** _RESCALE_BITS
            if np.any(big):
                cur[:l + 1] = np.where(big, np.ldexp(cur[:l + 1], -_RESCALE_BITS), cur[:l + 1])
                prev[:l + 1] = np.where(big, np.ldexp(prev[:l + 1], -_RESCALE_BITS), prev[:l + 1])
                e[:l + 1] = e[:l + 1] + np.where(big, _RESCALE_BITS, 0)
        yield l, np.ldexp(cur[:l + 1], e[:l + 1])
