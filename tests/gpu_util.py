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
