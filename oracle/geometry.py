"""HEALPix point set in RING order (oracle; test infrastructure only).

Follows eq. (healpts), Sec. 2.1 of the paper: 4*Nside-1 rings of constant
colatitude theta, numbered r = 1 .. 4*Nside-1 from the north pole.

  north cap, r = j < Nside:   cos(theta) = 1 - j^2/(3 Nside^2),
                              4j points at lambda = pi (k + 1/2) / (2j)
  equatorial, Nside <= r <= 3 Nside:
                              cos(theta) = 2 (2 Nside - r) / (3 Nside),
                              4 Nside points at
                              lambda = pi (k + ((r + 1) mod 2)/2) / (2 Nside)
  south cap, r = 4 Nside - j: cos(theta) = -(1 - j^2/(3 Nside^2)),
                              4j points at lambda = pi (k + 1/2) / (2j)

theta is the colatitude (the paper calls it latitude in places but defines it
through z = cos(theta), eq. (latlon)).  Pixels within a ring are stored with k
ascending; rings are stored north to south.  For even Nside this is the
standard RING ordering; Nside = 1 is not supported.

Parity pinned by: pixel counts, the z -> -z and lambda -> lambda + pi/2 maps
of the point set onto itself, and Table 1 (through the dense synthesis matrix).
"""

import numpy as np


def npix(nside):
    """N = 12 Nside^2 (Sec. 2.1)."""
    return 12 * nside * nside


def ring_table(nside):
    """Per-ring geometry for rings r = 1 .. 4 Nside - 1 (stored at index r-1).

    Returns a dict of numpy arrays:
      z      cos(theta_r)
      one_minus_abs_z  1 - |z| (exact form j^2 / (3 Nside^2) on the caps)
      theta  theta_r (colatitude), 2 arcsin(sqrt((1 - |z|)/2)) or pi minus it
      n      number of points on the ring
      phi0   longitude of the first point
      start  index of the first pixel of the ring in the RING-ordered map
    """
    if nside < 2 or (nside & (nside - 1)) != 0:
        raise ValueError("nside must be a power of two >= 2")
    nr = 4 * nside - 1
    z = np.empty(nr)
    omz = np.empty(nr)                     # 1 - |z|, from its exact form (no cancellation)
    n = np.empty(nr, dtype=np.int64)
    phi0 = np.empty(nr)
    ns2 = 3.0 * nside * nside
    for r in range(1, nr + 1):
        if r < nside:                      # north polar cap, j = r
            j = r
            omz[r - 1] = j * j / ns2
            z[r - 1] = 1.0 - omz[r - 1]
            n[r - 1] = 4 * j
            phi0[r - 1] = np.pi * 0.5 / (2 * j)
        elif r <= 3 * nside:               # equatorial belt
            z[r - 1] = 2.0 * (2 * nside - r) / (3.0 * nside)
            omz[r - 1] = 1.0 - abs(z[r - 1])
            n[r - 1] = 4 * nside
            phi0[r - 1] = np.pi * (((r + 1) % 2) / 2.0) / (2 * nside)
        else:                              # south polar cap, j = 4 Nside - r
            j = 4 * nside - r
            omz[r - 1] = j * j / ns2
            z[r - 1] = -(1.0 - omz[r - 1])
            n[r - 1] = 4 * j
            phi0[r - 1] = np.pi * 0.5 / (2 * j)
    start = np.zeros(nr, dtype=np.int64)
    start[1:] = np.cumsum(n)[:-1]
    # theta from 1 - |z| (2 arcsin sqrt((1 - |z|) / 2) is well conditioned at
    # the poles, where arccos of the rounded z loses most digits)
    half = 2.0 * np.arcsin(np.sqrt(omz / 2.0))
    theta = np.where(z >= 0.0, half, np.pi - half)
    return {"z": z, "one_minus_abs_z": omz, "theta": theta, "n": n, "phi0": phi0, "start": start}


def pixel_angles(nside):
    """(theta, lambda) of every pixel, RING order, eq. (healpts)."""
    rt = ring_table(nside)
    theta = np.repeat(rt["theta"], rt["n"])
    lam = np.concatenate([rt["phi0"][i] + 2.0 * np.pi * np.arange(rt["n"][i]) / rt["n"][i]
                          for i in range(len(rt["n"]))])
    return theta, lam


def pixel_xyz(nside):
    """Cartesian unit vectors of the pixel centres, eq. (latlon)."""
    theta, lam = pixel_angles(nside)
    st = np.sin(theta)
    return np.stack([np.cos(lam) * st, np.sin(lam) * st, np.cos(theta)], axis=1)
