"""O_ref: one refinement round of HP2SPH in FP64 (oracle; test infrastructure only).

One step of eq. (uzawa), Sec. 2.2, with the analysis A := HP2SPH (O_plain)
and the synthesis S := exact synthesis (O_synth):
    a0 = A f,   r = f - S a0,   a1 = a0 + A r.
HP2SPH is not an exact inverse of synthesis (a polar ring with 4j points
aliases longitude modes |m| >= 2j), so a1 differs from a0 even in exact
arithmetic; a1 is what an FP32 analysis plus one FP64-residual round tends to.

Parity: inherits the pins of O_plain and O_synth; additionally pinned by
a1 = a0 when the input is exactly recovered by HP2SPH (Y_l^{+-1}).
"""

from .hp2sph import analyze
from .synth import synthesize


def analyze_refined(f, nside, lmax=None):
    p = 2 * nside
    lmax = p if lmax is None else int(lmax)
    a0 = analyze(f, nside, lmax)
    r = f - synthesize(a0, nside, lmax)
    return a0 + analyze(r, nside, lmax)
