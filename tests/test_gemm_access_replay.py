"""Host-side replay of the grouped GEMM's memory accesses (no GPU): every
problem list a plan launches, at the benchmark shapes, stays inside its table
and workspace allocations, and every element the kernel stages is either read
in range or turned into a zero by the buffer descriptor's range check.  The
replay runs the kernel's own offset functions (kernels.h) through
hp2sph_gemm_check."""

import ctypes

import pytest

import paper_1904_10514_amd as P

CASES = [
    # the nside-1024 benchmark (per-order tables): analysis, refinement, equal weight
    (1024, 64, "f32_refine", "tables"),
    (1024, 64, "f64", "tables"),
    (1024, 64, "equal_weight", "tables"),
    # nside 2048, 16 maps (staged: four parity-block problems per GEMM)
    (2048, 16, "f32_refine", "staged"),
    (2048, 16, "f64", "staged"),
    (2048, 16, "equal_weight", "staged"),
    # the uneven batch's nside classes (per-order tables) and ragged small shapes
    (512, 73, "f32_refine", "tables"),
    (256, 52, "f32_refine", "tables"),
    (128, 73, "f32_refine", "tables"),
    (64, 58, "f32_refine", "tables"),
    (128, 3, "f32_refine", "staged"),
    (128, 3, "f32", "tables"),
    (16, 1, "f64", "tables"),
    (2, 1, "f32_refine", "staged"),
]


@pytest.mark.parametrize("nside,nmaps,mode,strategy", CASES)
def test_gemm_accesses_stay_in_bounds(nside, nmaps, mode, strategy):
    lib = P.lib()
    checked, bad, pad = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    rc = lib.hp2sph_gemm_check(nside, nmaps, P.MODES[mode], P.STRATEGIES[strategy], ctypes.byref(checked),
                               ctypes.byref(bad), ctypes.byref(pad))
    assert rc == 0, lib.hp2sph_last_error()
    print(f"{nside} x {nmaps} {mode} {strategy}: {checked.value} checks, {pad.value} padding reads")
    assert checked.value > 0
    assert bad.value == 0, lib.hp2sph_last_error().decode()
