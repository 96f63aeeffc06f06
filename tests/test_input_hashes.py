"""The seeded inputs stay what the recipes say (workloads/): SHA-256 of the
generator-exact draws against tests/golden/input_sha256.txt (written by
tests/golden/make_input_hashes.py), and the power spectra of every
configuration against their formulas (exp-based, so compared to a tolerance)."""

import importlib.util
import os

import numpy as np
import pytest

import workloads as W

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _maker():
    spec = importlib.util.spec_from_file_location("make_input_hashes", os.path.join(GOLD, "make_input_hashes.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_seeded_draws_match_their_recorded_hashes():
    mk = _maker()
    rows = [l.split(None, 1) for l in open(os.path.join(GOLD, "input_sha256.txt")) if l.strip() and l[0] != "#"]
    recorded = {label.strip(): h for h, label in rows}
    got = {label: mk.digest(arr) for label, arr in mk.entries()}
    assert set(got) == set(recorded)
    for label, h in got.items():
        assert h == recorded[label], label


@pytest.mark.parametrize("cid", [0, 1, 2, 3, 4])
def test_spectra_follow_their_formulas(cid):
    lmax = W.CONFIGS[cid]["lmax"] or 1024
    cl = W.spectrum(cid, lmax)
    l = np.arange(2, lmax + 1, dtype=np.float64)
    base = 1.0 / (l * (l + 1.0))
    if cid == 0:
        want = base
    elif cid in (1, 2):
        want = base * np.exp(-l * (l + 1.0) * 0.005 ** 2)
    elif cid == 3:
        want = np.exp(-l * (l + 1.0) * 0.005 ** 2) / l ** 2
    else:
        want = base * (1.0 + 4.0 * np.exp(-(l - 220.0) ** 2 / 7200.0)) * np.exp(-l * (l + 1.0) * 0.002 ** 2)
    assert cl[0] == 0.0 and cl[1] == 0.0
    np.testing.assert_allclose(cl[2:], want, rtol=1e-13, atol=0.0)
    if cid == 4:   # the bump is five times the baseline at l = 220
        i = 220 - 2
        assert cl[2:][i] / (base[i] * np.exp(-220 * 221 * 0.002 ** 2)) == pytest.approx(5.0, rel=1e-14)


def test_draws_have_the_stated_variance():
    lmax = 512
    a = W.draw_alm(np.ones(lmax + 1), lmax, W.rng_for(1, 0))
    m0 = a[:lmax + 1]
    assert np.all(m0.imag == 0.0)
    rest = a[lmax + 1:]
    nz = rest[rest != 0]
    # Re, Im ~ N(0, 1/2) for m >= 1, so E|a|^2 = 1 (about 130,000 draws)
    assert abs(np.mean(np.abs(nz) ** 2) - 1.0) < 0.02
    assert abs(np.mean(m0.real ** 2) - 1.0) < 0.2
