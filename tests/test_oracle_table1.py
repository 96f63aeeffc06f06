"""Table 1 of the paper as a pin of geometry + Y_l^m normalisation + dense S."""

import os

import numpy as np
import pytest

from oracle.dense import richardson_radius_readings

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1.txt")


def _table1():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                ns, n, v = line.split()
                rows.append((int(ns), int(n), float(v)))
    return rows


@pytest.mark.parametrize("nside,N,value", _table1())
def test_table1_printed_values(nside, N, value):
    assert 12 * nside * nside == N
    lam_max_minus_1, one_minus_lam_min = richardson_radius_readings(nside, 2 * nside)
    # printed to 4 decimals
    assert round(lam_max_minus_1, 4) == pytest.approx(value, abs=1e-12)
    # the other reading of the caption does not reproduce the printed values
    assert abs(one_minus_lam_min - value) > 1e-2


def test_table1_other_band_limit_does_not_reproduce():
    """lmax = 3 Nside - 1 (the HEALPix default) gives different numbers."""
    a, b = richardson_radius_readings(4, 11)
    assert abs(a - 0.0932) > 1e-2 and abs(b - 0.0932) > 1e-2
