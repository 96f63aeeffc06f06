"""FP64 CPU oracle for HP2SPH spherical-harmonic analysis on HEALPix grids.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or link anything in this package; only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark use it.
It shares no code, tables or helpers with the GPU path.

Everything here is plain, slow and written to be checked against the paper
(Drake & Wright, "A Fast and Accurate Algorithm for Spherical Harmonic
Analysis on HEALPix Grids ...", arXiv:1904.10514) by eye:

  geometry   -- the HEALPix point set, eq. (healpts), Sec. 2.1
  legendre   -- orthonormal associated Legendre functions and Y_l^m,
                Appendix A, eqs. (ssph), (sphip)
  hp2sph     -- O_plain: Algorithm 1 (HP2SPH) step by step, Sec. 3
  synth      -- O_synth: exact synthesis, eq. (synthesis), Sec. 2.2
  dense      -- O_dense: least squares against the dense Y matrix, and the
                Richardson matrix of eq. (richardson) (Table 1)
  refine     -- O_ref: one step of eq. (uzawa) with A := HP2SPH
  healpix    -- the equal-weight analysis of eq. (healsph) and its Jacobi
                iteration, eq. (uzawa) with A := (4 pi / N) S^*, Sec. 2.2
  spectrum   -- the angular power spectrum, eq. (APS), Sec. 1

Parity status of each function is stated in its docstring.
"""

from .geometry import ring_table, pixel_angles, npix
from .legendre import plm_orthonormal, ylm, gauss_legendre
from .hp2sph import analyze, analyze_full, analyze_columns, ring_coefficients, pole_values
from .synth import synthesize
from .dense import synthesis_matrix, analyze_dense, richardson_radius_readings
from .refine import analyze_refined
from .healpix import analyze_equal_weight, analyze_jacobi, ring_longitude_sums, equal_weight_columns
from .spectrum import power_spectrum, alm_index, alm_size

__all__ = [
    "ring_table", "pixel_angles", "npix",
    "plm_orthonormal", "ylm", "gauss_legendre",
    "analyze", "analyze_full", "analyze_columns", "ring_coefficients", "pole_values",
    "synthesize",
    "synthesis_matrix", "analyze_dense", "richardson_radius_readings",
    "analyze_refined",
    "analyze_equal_weight", "analyze_jacobi", "ring_longitude_sums", "equal_weight_columns",
    "power_spectrum", "alm_index", "alm_size",
]
