"""Writes tests/golden/input_sha256.txt: SHA-256 of the seeded random draws
every workload starts from (workloads/), so that a change to a recipe, a seed
or the generator shows up as a failing CPU test.

Only results of exact arithmetic on the generator's output are hashed
(little-endian bytes), so the hashes are the same on every host: the a_lm of
map 0 of each configuration drawn with a unit spectrum (the draw order and
layout of draw_alm, scaled by sqrt(1/2) only) and, for configuration 0, with
its own spectrum 1/(l(l+1)) (divisions and square roots, correctly rounded);
the white-noise maps the parity tests use; the nside list of the uneven batch.
The exp-based spectra of the other configurations are checked against their
formulas with a tolerance instead (tests/test_input_hashes.py), and maps
synthesised from the draws go through floating-point transforms whose last
bits may differ between hosts; the benchmark records the hash of the map it
times.

Usage (repository root): python tests/golden/make_input_hashes.py
"""

import hashlib
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import workloads as W   # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "input_sha256.txt")


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).astype(a.dtype.newbyteorder("<")).tobytes()).hexdigest()


def entries():
    """(label, array) pairs, in file order."""
    out = []
    lmax0 = W.CONFIGS[0]["lmax"]
    out.append((f"alm config=0 map=0 lmax={lmax0}", W.draw_alm(W.spectrum(0, lmax0), lmax0, W.rng_for(0, 0))))
    nsides = W.uneven_nsides(256, 3)
    out.append(("uneven_nsides config=3 batch=256", np.asarray(nsides, dtype=np.int64)))
    for cid in (0, 1, 2, 3, 4):
        lmax = W.CONFIGS[cid]["lmax"] or 2 * int(nsides[0])
        out.append((f"unit-spectrum alm config={cid} map=0 lmax={lmax}",
                    W.draw_alm(np.ones(lmax + 1), lmax, W.rng_for(cid, 0))))
    for nside, seed in ((16, 0), (64, 1)):
        out.append((f"white_map nside={nside} rng=(99,{seed})", W.random_map(12 * nside * nside, W.rng_for(99, seed))))
    return out


def main():
    with open(OUT, "w") as fh:
        fh.write("# SHA-256 of the seeded draws of workloads/ (written by make_input_hashes.py)\n")
        for label, arr in entries():
            fh.write(f"{digest(arr)}  {label}\n")
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
