"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds only random draws and spectrum recipes -- none of the
analysis or synthesis arithmetic -- so the oracle and the GPU path can both be
fed from it without sharing any of the method.

Recipes (all seeded through SeedSequence([1904, 10514, config_id, map_index])):

  config 0  one map, nside 16, lmax 32;   C_l = 1/(l(l+1)), l >= 2
  config 1  one map, nside 256, lmax 512; C_l = exp(-l(l+1) s^2)/(l(l+1)), s = 0.005
  config 2  64 maps, nside 1024, lmax 2048; as config 1, plus white pixel noise
            of standard deviation 1e-3 times the signal rms
  config 3  256 maps, nside drawn uniformly from {64, 128, 256, 512},
            lmax = 2 nside; C_l = l^-2 exp(-l(l+1) s^2), s = 0.005
  config 4  16 maps, nside 2048, lmax 4096;
            C_l = [1/(l(l+1))] [1 + 4 exp(-(l-220)^2/(2*60^2))] exp(-l(l+1) s^2),
            s = 0.002 (a bump five times the baseline at l = 220, width 60)

a_l^0 ~ N(0, C_l) (real); for m >= 1 Re and Im ~ N(0, C_l/2); a_0^0 = a_1^m = 0.
Coefficients are packed m-major for m >= 0: index m (2 lmax + 1 - m)/2 + l.
"""

import numpy as np

SEED_ROOT = (1904, 10514)

CONFIGS = {
    0: {"name": "nside16_L32_f64", "nside": 16, "lmax": 32, "batch": 1},
    1: {"name": "nside256_L512_f64", "nside": 256, "lmax": 512, "batch": 1},
    2: {"name": "nside1024_L2048_b64", "nside": 1024, "lmax": 2048, "batch": 64},
    3: {"name": "uneven_b256_nside64to512", "nside": None, "lmax": None, "batch": 256},
    4: {"name": "nside2048_L4096_b16", "nside": 2048, "lmax": 4096, "batch": 16},
}


def rng_for(config_id, map_index):
    return np.random.default_rng(np.random.SeedSequence([*SEED_ROOT, int(config_id), int(map_index)]))


def spectrum(config_id, lmax):
    """C_l for l = 0 .. lmax (C_0 = C_1 = 0)."""
    l = np.arange(lmax + 1, dtype=np.float64)
    cl = np.zeros(lmax + 1)
    ll = l[2:] * (l[2:] + 1.0)
    if config_id == 0:
        cl[2:] = 1.0 / ll
    elif config_id in (1, 2):
        cl[2:] = np.exp(-ll * 0.005 ** 2) / ll
    elif config_id == 3:
        cl[2:] = l[2:] ** -2.0 * np.exp(-ll * 0.005 ** 2)
    elif config_id == 4:
        bump = 1.0 + 4.0 * np.exp(-(l[2:] - 220.0) ** 2 / (2.0 * 60.0 ** 2))
        cl[2:] = bump / ll * np.exp(-ll * 0.002 ** 2)
    else:
        raise ValueError("unknown config")
    return cl


def alm_size(lmax):
    return (lmax + 1) * (lmax + 2) // 2


def draw_alm(cl, lmax, rng):
    """Gaussian a_l^m with variance C_l, packed m-major (m >= 0)."""
    out = np.zeros(alm_size(lmax), dtype=np.complex128)
    for m in range(lmax + 1):
        base = m * (2 * lmax + 1 - m) // 2
        c = cl[m:lmax + 1]
        if m == 0:
            out[base:base + lmax + 1] = rng.standard_normal(lmax + 1) * np.sqrt(c)
        else:
            re = rng.standard_normal(lmax + 1 - m)
            im = rng.standard_normal(lmax + 1 - m)
            out[base + m:base + lmax + 1] = (re + 1j * im) * np.sqrt(c / 2.0)
    return out


def uneven_nsides(batch=256, config_id=3):
    """nside per map for the uneven batch, uniform over {64, 128, 256, 512}."""
    rng = rng_for(config_id, 1 << 20)
    return rng.choice(np.array([64, 128, 256, 512]), size=batch)


def white_noise(npix, sigma, rng):
    return rng.standard_normal(npix) * sigma


def random_map(npix, rng):
    """A map of independent standard-normal pixels (all scales present)."""
    return rng.standard_normal(npix)
