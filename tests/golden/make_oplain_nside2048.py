"""Writes tests/golden/oplain_nside2048.txt: the FP64 oracle's HP2SPH analysis
(O_plain, Algorithm 1, by the order-by-order route of the Remark of
Sec. 3.2.1) of one seeded white-noise map at the largest supported size,
nside 2048, lmax 4096, for the full-size test of the staged strategy
(tests/test_gpu_maxsize.py).

Map: seeded standard-normal pixels, SeedSequence([1904, 10514, 14, 0]) (every
scale present, so every order carries data).  Stored: the map's SHA-256
(its draws are exact on every host, tests/golden/make_input_hashes.py) and
a_l^m for the sampled orders ORDERS at the degrees sampled_degrees(m) (the
first and last 8 of the order and every 32nd in between).

Only oracle/ and workloads/ are called.  Takes about 10 minutes on 8 cores
(most of it the dense QR of the 16384 x 8193 colatitude fit).

Usage (repository root): python tests/golden/make_oplain_nside2048.py
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oplain_nside2048.txt")
NSIDE, LMAX = 2048, 4096
ORDERS = (0, 1, 2, 3, 5, 64, 1000, 2047, 2048, 3001, 4095, 4096)


def sampled_degrees(m):
    ls = set(range(m, min(m + 8, LMAX + 1))) | set(range(max(m, LMAX - 7), LMAX + 1)) | set(range(m, LMAX + 1, 32))
    return sorted(ls)


def white_map():
    return W.random_map(O.npix(NSIDE), W.rng_for(14, 0))


def main():
    t0 = time.time()
    f = white_map()
    cols = O.analyze_columns(f, NSIDE, list(ORDERS), LMAX)
    print(f"O_plain on {len(ORDERS)} orders in {time.time() - t0:.0f} s", flush=True)
    lines = ["# FP64 oracle (O_plain, order-by-order route) at nside 2048, lmax 4096, one white-noise map",
             "# written by tests/golden/make_oplain_nside2048.py",
             "sha256 " + hashlib.sha256(np.ascontiguousarray(f).astype("<f8").tobytes()).hexdigest()]
    for m in ORDERS:
        col = cols[m]                                  # l = m .. LMAX
        for l in sampled_degrees(m):
            v = col[l - m]
            lines.append(f"alm {m} {l} {v.real:.17e} {v.imag:.17e}")
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
