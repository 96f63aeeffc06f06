"""Writes tests/golden/oref_nside1024.txt: the FP64 oracle's HP2SPH analysis
(O_plain, Algorithm 1) and its refined variant (O_ref, one step of eq. uzawa of
Sec. 2.2 with A := HP2SPH and S := exact synthesis) of two maps of the
benchmark's shape (nside 1024, lmax 2048), for the full-size accuracy test of
the FP32 + refinement analysis (tests/test_gpu_headline_accuracy.py).

Maps (both rebuilt by the test with the same calls):
  cmb    the a_lm of map 0 of the nside-1024 workload (workloads config 2:
         C_l = exp(-l(l+1) s^2) / (l(l+1)), s = 0.005) through the oracle's
         exact synthesis, plus white pixel noise of standard deviation
         1e-3 x the synthesised map's rms, drawn from
         SeedSequence([1904, 10514, 2, 65536]);
  white  seeded standard-normal pixels (SeedSequence([1904, 10514, 9, 0]), map
         0 of the white-noise batch of tests/test_gpu_fullsize.py): every
         scale present, the input on which I - A S is largest.

Stored per map: the map's SHA-256 and checksums (sum and sum of squares, to
compare a rebuilt map whose last bits may differ on another host), C_l for
l = 0..2048 of O_plain and O_ref (eq. APS), and a_l^m of O_plain and O_ref for
the sampled orders ORDERS at the degrees sampled_degrees(m) (the first and
last 8 of the order and every 16th in between).

Only oracle/ and workloads/ are called.  Takes about 15 minutes on 8 cores.

Usage (repository root): python tests/golden/make_oref_nside1024.py
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oref_nside1024.txt")
NSIDE, LMAX = 1024, 2048
ORDERS = (0, 1, 2, 3, 8, 64, 512, 1024, 2000, 2048)
NOISE_STREAM = 1 << 16


def sampled_degrees(m):
    ls = set(range(m, min(m + 8, LMAX + 1))) | set(range(max(m, LMAX - 7), LMAX + 1)) | set(range(m, LMAX + 1, 16))
    return sorted(ls)


def cmb_map():
    a = W.draw_alm(W.spectrum(2, LMAX), LMAX, W.rng_for(2, 0))
    f = O.synthesize(a, NSIDE, LMAX)
    rms = float(np.sqrt(np.mean(f * f)))
    return f + W.white_noise(f.size, 1e-3 * rms, W.rng_for(2, NOISE_STREAM))


def white_map():
    return W.random_map(O.npix(NSIDE), W.rng_for(9, 0))


def sha(f):
    return hashlib.sha256(np.ascontiguousarray(f).astype("<f8").tobytes()).hexdigest()


def main():
    lines = ["# FP64 oracle at nside 1024, lmax 2048 (written by tests/golden/make_oref_nside1024.py)",
             "# orders " + " ".join(str(m) for m in ORDERS)]
    for name, build in (("cmb", cmb_map), ("white", white_map)):
        t0 = time.time()
        f = build()
        print(f"{name}: map built in {time.time() - t0:.0f} s", flush=True)
        a0 = O.analyze(f, NSIDE, LMAX)
        print(f"{name}: O_plain in {time.time() - t0:.0f} s", flush=True)
        r = f - O.synthesize(a0, NSIDE, LMAX)
        a1 = a0 + O.analyze(r, NSIDE, LMAX)
        print(f"{name}: O_ref in {time.time() - t0:.0f} s", flush=True)
        c0, c1 = O.power_spectrum(a0, LMAX), O.power_spectrum(a1, LMAX)
        lines.append(f"map {name}")
        lines.append(f"sha256 {sha(f)}")
        lines.append(f"checksum {np.sum(f):.17e} {np.sum(f * f):.17e}")
        for l in range(LMAX + 1):
            lines.append(f"cl {l} {c0[l]:.17e} {c1[l]:.17e}")
        for m in ORDERS:
            for l in sampled_degrees(m):
                i = O.alm_index(l, m, LMAX)
                lines.append(f"alm {m} {l} {a0[i].real:.17e} {a0[i].imag:.17e} {a1[i].real:.17e} {a1[i].imag:.17e}")
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
