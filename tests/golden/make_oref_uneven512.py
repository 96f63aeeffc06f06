"""Writes tests/golden/oref_uneven_nside512.txt: the FP64 oracle's refined
analysis O_ref (one step of eq. uzawa of Sec. 2.2 with A := HP2SPH, S :=
exact synthesis) of the first nside-512 map of the uneven batch (256 maps of
nside drawn from {64, 128, 256, 512}; the white-noise maps of
tests/test_gpu_uneven_fullsize.py), lmax 1024, for the FP32 + refinement
check of that test's largest class.

Map: seeded standard-normal pixels, SeedSequence([1904, 10514, 13, i]) with i
the batch index of the first nside-512 map.  Stored: i, the map's SHA-256, C_l
of O_ref for l = 0..1024 and a_l^m of O_ref for the sampled orders ORDERS at
the degrees sampled_degrees(m) (the first and last 8 of the order and every
16th in between).

Only oracle/ and workloads/ are called.  Takes about 2 minutes on 8 cores.

Usage (repository root): python tests/golden/make_oref_uneven512.py
"""

import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as O      # noqa: E402
import workloads as W   # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oref_uneven_nside512.txt")
NSIDE, LMAX = 512, 1024
ORDERS = (0, 1, 2, 3, 7, 100, 511, 512, 1000, 1023, 1024)


def sampled_degrees(m):
    ls = set(range(m, min(m + 8, LMAX + 1))) | set(range(max(m, LMAX - 7), LMAX + 1)) | set(range(m, LMAX + 1, 16))
    return sorted(ls)


def map_index():
    return [int(v) for v in W.uneven_nsides(256, 3)].index(NSIDE)


def white_map():
    return W.random_map(O.npix(NSIDE), W.rng_for(13, map_index()))


def main():
    t0 = time.time()
    f = white_map()
    a1 = O.analyze_refined(f, NSIDE, LMAX)
    print(f"O_ref in {time.time() - t0:.0f} s", flush=True)
    cl = O.power_spectrum(a1, LMAX)
    lines = ["# FP64 oracle (O_ref) at nside 512, lmax 1024: first nside-512 map of the uneven batch",
             "# written by tests/golden/make_oref_uneven512.py",
             f"index {map_index()}",
             "sha256 " + hashlib.sha256(np.ascontiguousarray(f).astype("<f8").tobytes()).hexdigest()]
    lines += [f"cl {l} {cl[l]:.17e}" for l in range(LMAX + 1)]
    for m in ORDERS:
        for l in sampled_degrees(m):
            v = a1[O.alm_index(l, m, LMAX)]
            lines.append(f"alm {m} {l} {v.real:.17e} {v.imag:.17e}")
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
