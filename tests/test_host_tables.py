"""Host logic of libhp2sph (no GPU): C-ABI surface, error paths, set-up tables.

The set-up tables are checked by emulating the staged GPU algorithm with them
in numpy (ring spectra from the oracle's Step 1, north/south sums, the four
parity blocks, the Givens sweeps) and comparing with the oracle's end result.
"""

import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
from oracle import hp2sph as OH
from oracle.geometry import ring_table
from oracle.legendre import gauss_legendre, plm_orthonormal

import paper_1904_10514_amd as P

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "hp2sph.h")


def test_library_exports_every_declared_symbol():
    names = set(re.findall(r"\b(hp2sph_[a-z_]+)\s*\(", open(HEADER).read()))
    assert names, "no declarations found"
    lib = P.lib()
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert names == set(P.EXPORTED)


def test_error_paths_without_gpu():
    lib = P.lib()
    h = ctypes.c_void_p()
    one = (ctypes.c_int32 * 1)(3)            # not a power of two
    lm = (ctypes.c_int32 * 1)(6)
    assert lib.hp2sph_plan_create(one, lm, 1, 0, ctypes.byref(h)) == -1
    assert b"power of two" in lib.hp2sph_last_error()
    two = (ctypes.c_int32 * 1)(8)
    big = (ctypes.c_int32 * 1)(17)           # lmax > 2 nside
    assert lib.hp2sph_plan_create(two, big, 1, 0, ctypes.byref(h)) == -1
    assert lib.hp2sph_plan_create(two, lm, 1, 7, ctypes.byref(h)) == -1      # bad mode
    assert lib.hp2sph_plan_create(two, lm, 0, 0, ctypes.byref(h)) == -1      # empty batch
    assert lib.hp2sph_plan_create(two, lm, 1, 0, None) == -1
    ws = ctypes.c_size_t()
    assert lib.hp2sph_workspace_size(None, ctypes.byref(ws)) == -5
    assert lib.hp2sph_analyze(None, None, None, None, 0, None) == -5
    assert lib.hp2sph_synthesize(None, None, None, None, 0, None) == -5
    assert lib.hp2sph_power_spectrum(None, None, None, None) == -5
    assert lib.hp2sph_plan_destroy(None) == -5
    assert lib.hp2sph_analyze_iterative(None, None, None, 3, None, 0, None) == -5
    # a handle that was never created is looked up among the live plans and
    # refused without being read through (here: the address of a host buffer)
    fake = ctypes.create_string_buffer(4096)
    fh = ctypes.cast(fake, ctypes.c_void_p)
    assert lib.hp2sph_plan_destroy(fh) == -5
    assert b"live plan" in lib.hp2sph_last_error()
    assert lib.hp2sph_workspace_size(fh, ctypes.byref(ws)) == -5
    assert lib.hp2sph_analyze(fh, None, None, None, 0, None) == -5
    assert fake.raw == bytes(4096)
    st = ctypes.c_int32()
    assert lib.hp2sph_plan_strategy(None, ctypes.byref(st)) == -5
    assert lib.hp2sph_profile(None, 1) == -5
    ms = (ctypes.c_double * P.NSTAGES)()
    nl = (ctypes.c_int32 * P.NSTAGES)()
    assert lib.hp2sph_profile_read(None, ms, nl, P.NSTAGES) == -5
    assert lib.hp2sph_plan_create_ex(two, lm, 1, 0, 9, ctypes.byref(h)) == -1          # bad strategy
    assert b"strategy" in lib.hp2sph_last_error()
    for bad_nside in (1, 2 * P.MAX_NSIDE):
        ns = (ctypes.c_int32 * 1)(bad_nside)
        assert lib.hp2sph_plan_create(ns, lm, 1, 0, ctypes.byref(h)) == -1
    neg = (ctypes.c_int32 * 1)(-1)
    assert lib.hp2sph_plan_create(two, neg, 1, P.HP2SPH_EQUAL_WEIGHT, ctypes.byref(h)) == -1
    assert b"lmax" in lib.hp2sph_last_error()
    # a batch is rejected as a whole if any map is invalid
    mixed_n = (ctypes.c_int32 * 3)(8, 16, 12)
    mixed_l = (ctypes.c_int32 * 3)(16, 32, 24)
    assert lib.hp2sph_plan_create(mixed_n, mixed_l, 3, 0, ctypes.byref(h)) == -1
    assert not h.value
    cnt = ctypes.c_int64()
    assert lib.hp2sph_host_table(12, 0, 0, None, 0, ctypes.byref(cnt)) == -1
    assert lib.hp2sph_host_table(8, 9, 0, None, 0, ctypes.byref(cnt)) == -1
    assert lib.hp2sph_host_table(8, 2, 4, None, 0, ctypes.byref(cnt)) == -1


@pytest.mark.parametrize("nside", [2, 8, 64])
def test_ring_table_matches_oracle_geometry(nside):
    t = P.host_table(nside, P.TABLE_RINGS).reshape(-1, 4)
    rt = ring_table(nside)
    np.testing.assert_allclose(t[:, 0], rt["z"], atol=1e-15)
    assert np.array_equal(t[:, 1].astype(int), rt["n"])
    np.testing.assert_allclose(t[:, 2], rt["phi0"], atol=1e-15)
    assert np.array_equal(t[:, 3].astype(int), rt["start"])


@pytest.mark.parametrize("nside", [2, 4, 32])
def test_pole_weights_reproduce_oracle_pole_values(nside):
    f = np.random.default_rng(11).standard_normal(O.npix(nside))
    w = P.host_table(nside, P.TABLE_POLE)
    rt = ring_table(nside)
    nr = len(rt["n"])
    mean = lambda r: f[rt["start"][r]:rt["start"][r] + rt["n"][r]].mean()
    fn = sum(w[i] * mean(i) for i in range(3))
    fs = sum(w[i] * mean(nr - 1 - i) for i in range(3))
    on, os_ = OH.pole_values(f, nside)
    assert fn == pytest.approx(on, abs=1e-12)
    assert fs == pytest.approx(os_, abs=1e-12)


@pytest.mark.parametrize("l,mp", [(2, 2), (3, 3), (4, 2), (9, 4), (30, 7), (200, 150), (513, 6)])
def test_givens_angles_against_quadrature(l, mp):
    """s = <Pt_l^m', Pt_l^{m'-2}> (closed form) and c = <Pt_{l-2}^{m'-2} ..>: pin P7."""
    nq = l + 2
    x, wq = gauss_legendre(nq)
    a = plm_orthonormal(l, mp, x)[l - mp]
    b = plm_orthonormal(l, mp - 2, x)[l - mp + 2]
    s_quad = np.sum(wq * a * b)
    blk = 0 if (mp % 2 == 0 and (l - mp) % 2 == 0) else None
    # read the table entry for this (l, m') from the right block
    kpar = mp % 2
    for b_ in (2 * kpar, 2 * kpar + 1):
        lmin = [0, 1, 1, 2][b_]
        if (l - lmin) % 2 == 0:
            blk = b_
    nside = 512
    lp, t = (l - [0, 1, 1, 2][blk]) // 2, (mp - kpar) // 2
    g = P.host_table(nside, P.TABLE_GIVENS, blk)
    nl = (2 * nside - [0, 1, 1, 2][blk]) // 2 + 1
    c, s = g[((t - 1) * nl + lp) * 2], g[((t - 1) * nl + lp) * 2 + 1]
    assert s == pytest.approx(s_quad, abs=1e-13)
    assert c * c + s * s == pytest.approx(1.0, abs=1e-15)
    assert c > 0 and s < 0


def _ring_D(f, nside):
    """D_r[k], k = 0..p, of the upsampled rows (oracle Step 1 + Nyquist fold)."""
    p = 2 * nside
    coefs = OH.ring_coefficients(f, nside)
    D = np.zeros((len(coefs), p + 1), dtype=np.complex128)
    for r, c in enumerate(coefs):
        n = len(c) - 1
        ks = np.arange(-n // 2, n // 2 + 1)
        for k in range(p + 1):
            sel = (ks == k) if k < p else ((ks == p) | (ks == -p))
            v = np.sum(c[sel])
            D[r, k] = v if k < p else 0.5 * v
    return D


def emulate_analysis(f, nside):
    """The staged algorithm with the library's host tables, in numpy."""
    p = 2 * nside
    K = 2 * nside + 1
    D = _ring_D(f, nside)
    nr = D.shape[0]
    Dp = np.zeros((K, p + 1), dtype=np.complex128)
    Dm = np.zeros_like(Dp)
    for h in range(1, 2 * nside):
        Dp[h] = 0.5 * (D[h - 1] + D[nr - h])
        Dm[h] = 0.5 * (D[h - 1] - D[nr - h])
    Dp[2 * nside] = D[2 * nside - 1]
    w = P.host_table(nside, P.TABLE_POLE)
    Dp[0, 0] = sum(w[i] * Dp[i + 1, 0] for i in range(3))
    Dm[0, 0] = sum(w[i] * Dm[i + 1, 0] for i in range(3))
    out = {}
    for b in range(4):
        kpar, sym = b >> 1, b & 1
        lmin = [0, 1, 1, 2][b]
        nl = (p - lmin) // 2 + 1
        A = P.host_table(nside, P.TABLE_ANALYSIS, b).reshape(K, nl)
        G = P.host_table(nside, P.TABLE_GIVENS, b)
        T = G.size // (2 * nl)
        G = G.reshape(T, nl, 2) if T else G
        src = Dp if sym == 0 else Dm
        for m in range(kpar, p + 1, 2):
            kk = m // 2
            x = A.T @ src[:, m]
            for t in range(1, kk + 1):
                carry = x[t - 1]
                for lp in range(t, nl):
                    c, s = G[t - 1, lp]
                    xo = x[lp]
                    x[lp] = c * carry + s * xo
                    carry = -s * carry + c * xo
            for lp in range(kk, nl):
                l = lmin + 2 * lp
                if l >= m:
                    out[(l, m)] = x[lp]
    return out


@pytest.mark.parametrize("nside", [2, 4, 16])
def test_tables_reproduce_the_oracle_through_the_staged_algorithm(nside):
    f = np.random.default_rng(12).standard_normal(O.npix(nside))
    ref = O.analyze(f, nside)
    em = emulate_analysis(f, nside)
    p = 2 * nside
    assert len(em) == O.alm_size(p)
    err = max(abs(v - ref[O.alm_index(l, m, p)]) for (l, m), v in em.items())
    assert err < 1e-13


@pytest.mark.parametrize("nside", [4, 16])
def test_synthesis_tables_reproduce_oracle_synthesis(nside):
    """Reverse sweeps + evaluation matrices + per-ring fold reproduce O_synth."""
    p = 2 * nside
    K = 2 * nside + 1
    rng = np.random.default_rng(13)
    a = rng.standard_normal(O.alm_size(p)) + 1j * rng.standard_normal(O.alm_size(p))
    Dp = np.zeros((K, p + 1), dtype=np.complex128)
    Dm = np.zeros_like(Dp)
    for b in range(4):
        kpar, sym = b >> 1, b & 1
        lmin = [0, 1, 1, 2][b]
        nl = (p - lmin) // 2 + 1
        E = P.host_table(nside, P.TABLE_SYNTHESIS, b).reshape(nl, K)
        G = P.host_table(nside, P.TABLE_GIVENS, b)
        T = G.size // (2 * nl)
        G = G.reshape(T, nl, 2) if T else G
        for m in range(kpar, p + 1, 2):
            kk = m // 2
            x = np.zeros(nl, dtype=np.complex128)
            for lp in range(nl):
                l = lmin + 2 * lp
                if l >= m:
                    x[lp] = a[O.alm_index(l, m, p)]
            for t in range(kk, 0, -1):
                carry = 0.0
                for lp in range(nl - 1, t - 1, -1):
                    c, s = G[t - 1, lp]
                    xp = x[lp]
                    x[lp] = s * xp + c * carry
                    carry = c * xp - s * carry
                x[t - 1] = carry
            (Dp if sym == 0 else Dm)[:, m] = E.T @ x
    rt = ring_table(nside)
    nr = len(rt["n"])
    out = np.zeros(O.npix(nside))
    for r in range(nr):
        h = r + 1 if r < 2 * nside else nr - r
        D = Dp[h] + Dm[h] if r < 2 * nside else Dp[h] - Dm[h]
        n = rt["n"][r]
        H = np.zeros(n, dtype=np.complex128)
        k = np.arange(p + 1)
        g = D * np.exp(1j * k * rt["phi0"][r])
        np.add.at(H, k % n, g)
        np.add.at(H, (-k[1:]) % n, np.conj(g[1:]))
        out[rt["start"][r]:rt["start"][r] + n] = (np.fft.ifft(H) * n).real
    ref = O.synthesize(a, nside, p)
    assert np.max(np.abs(out - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_table_cache_round_trip_and_rejects_foreign_files(tmp_path, monkeypatch):
    """HP2SPH_TABLE_CACHE: the first build writes one file per nside, later
    builds read it back bit for bit; a truncated file or one with another
    build stamp is ignored (rebuilt and rewritten), never half-read."""
    monkeypatch.delenv("HP2SPH_TABLE_CACHE", raising=False)
    nside = 8
    fresh = {(t, b): P.host_table(nside, t, b) for t in (2, 3, 4) for b in range(4)}
    fresh[(1, 0)] = P.host_table(nside, 1, 0)
    monkeypatch.setenv("HP2SPH_TABLE_CACHE", str(tmp_path))
    path = tmp_path / f"hp2sph_tables_nside{nside}.bin"

    def all_equal():
        return all(np.array_equal(P.host_table(nside, t, b), v) for (t, b), v in fresh.items())

    assert all_equal()                      # builds and writes
    assert path.exists()
    size = path.stat().st_size
    assert all_equal()                      # reads
    # a truncated file: ignored, rebuilt, rewritten whole
    data = path.read_bytes()
    path.write_bytes(data[: size // 2])
    assert all_equal()
    assert path.stat().st_size == size
    # another build's stamp: ignored
    bad = bytearray(path.read_bytes())
    bad[8:40] = b"Jan  1 1970 00:00:00".ljust(32, b"\0")
    path.write_bytes(bytes(bad))
    assert all_equal()
    assert path.read_bytes() == data
    # the read path is what serves a cached nside: a value changed in the
    # file (the first entry of the block-0 analysis matrix, after the
    # 80-byte header and the ring table of 4 nside - 1 records of 40 bytes)
    # comes back as changed
    off = 80 + 8 + (4 * nside - 1) * 40 + 8
    assert data[off:off + 8] == fresh[(2, 0)][:1].tobytes()
    poisoned = bytearray(data)
    poisoned[off:off + 8] = np.float64(12345.0).tobytes()
    path.write_bytes(bytes(poisoned))
    got = P.host_table(nside, 2, 0)
    assert got[0] == 12345.0 and np.array_equal(got[1:], fresh[(2, 0)][1:])
