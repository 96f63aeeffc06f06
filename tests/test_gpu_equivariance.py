"""Exact equivariances of the HEALPix point set on the GPU at full size, every
order: the batch holds a map f and its images under three maps of the point
set onto itself, and the analysis must commute with them (Sec. 2.1, eq.
healpts; pinned on the oracle in tests/test_oracle_hp2sph.py):

  lambda -> lambda + pi/2 (every ring rolled by a quarter turn):
                        a_l^m -> e^{-i m pi/2} a_l^m
  z -> -z (ring r <-> ring 4 nside - r):   a_l^m -> (-1)^{l+m} a_l^m
  lambda -> -lambda (reflection of every ring):  a_l^m -> conj(a_l^m)

Each image is analysed in the same launch as f, so every per-order GEMM, the
Givens sweeps of the staged strategy, the residual fold's alias chains and the
synthesis of the refinement see non-zero data at every order m: a dropped or
misplaced tile at any order breaks an identity.  FP64 must commute to
rounding; FP32 + refinement to its own accuracy (the FP32 rounding differs
between a map and its image).  Maps: seeded CMB-like fields (the benchmark
recipes, synthesised on the GPU: these are GPU-against-GPU identities, no
oracle involved) plus seeded white noise (every scale present)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import oracle as O                  # noqa: E402
import workloads as W               # noqa: E402
import paper_1904_10514_amd as P    # noqa: E402

# FP64: both results carry up to kappa p eps of rounding (kappa <= 50, the
# condition number of the colatitude fit), with p = 2 nside;
# FP32 + refinement: each result is within ~1e-6 of max |a| of the exact
# refined value on white noise (tests/test_gpu_headline_accuracy.py)
def _tol(mode, nside):
    return 50 * 2 * nside * 1.1e-16 if mode == "f64" else 5e-6


def _images(f, nside):
    """f and its three images, each a (npix,) float64 torch tensor on the GPU."""
    rt = O.ring_table(nside)
    npix = O.npix(nside)
    roll = np.empty(npix, dtype=np.int64)
    swap = np.empty(npix, dtype=np.int64)
    refl = np.empty(npix, dtype=np.int64)
    nr = len(rt["n"])
    for r in range(nr):
        s, n = int(rt["start"][r]), int(rt["n"][r])
        q = np.arange(n)
        roll[s:s + n] = s + (q - n // 4) % n                     # g(q) = f(q - n/4): lambda -> lambda + pi/2
        t = int(rt["start"][nr - 1 - r])
        swap[s:s + n] = t + q                                      # ring r <- ring 4 nside - r
        refl[s:s + n] = s + ((-q) % n if rt["phi0"][r] == 0.0 else (-q - 1) % n)
    idx = [torch.from_numpy(v).cuda() for v in (roll, swap, refl)]
    return [f] + [f[i] for i in idx]


def _expected(a, lmax):
    """The three transformed coefficient sets of the packed m-major a (complex128, GPU)."""
    m = np.zeros(O.alm_size(lmax), dtype=np.int64)
    l = np.zeros_like(m)
    for mm in range(lmax + 1):
        b = mm * (2 * lmax + 1 - mm) // 2
        m[b + mm:b + lmax + 1] = mm
        l[b + mm:b + lmax + 1] = np.arange(mm, lmax + 1)
    md = torch.from_numpy(m).cuda()
    ld = torch.from_numpy(l).cuda()
    rot = torch.exp(-0.5j * np.pi * md.to(torch.float64))
    par = 1.0 - 2.0 * ((ld + md) % 2).to(torch.float64)
    return [a * rot, a * par, torch.conj(a)]


def _check(nside, mode, cfg, nwhite, seed):
    """A CMB-like map of workloads config `cfg` (synthesised on the GPU by the
    plan itself) and `nwhite` white-noise maps, each with its three images."""
    lmax = 2 * nside
    nbase = 1 + nwhite
    plan = P.Plan(nside, lmax, batch=4 * nbase, mode=mode)
    alm = np.zeros((4 * nbase, O.alm_size(lmax)), dtype=np.complex128)
    alm[0] = W.draw_alm(W.spectrum(cfg, lmax), lmax, W.rng_for(cfg, seed))
    cmb = plan.synthesize(torch.from_numpy(alm.reshape(-1)).cuda()).view(4 * nbase, -1)[0].clone()
    del alm
    npix = O.npix(nside)
    base = [cmb] + [torch.from_numpy(W.random_map(npix, W.rng_for(15, seed + v))).cuda() for v in range(nwhite)]
    dev = torch.cat([g for f in base for g in _images(f, nside)])
    del base, cmb
    a = plan.analyze(dev).view(4 * nbase, -1)
    torch.cuda.synchronize()
    tol = _tol(mode, nside)
    worst = 0.0
    for i in range(nbase):
        a0 = a[4 * i]
        scale = float(a0.abs().max())
        for j, e in enumerate(_expected(a0, lmax)):
            err = float((a[4 * i + 1 + j] - e).abs().max()) / scale
            worst = max(worst, err)
            assert err < tol, (i, j, err)
    print(f"nside {nside} {mode} ({plan.strategy}): worst equivariance error {worst:.3e} (bound {tol:.1e})")
    plan.close()


@pytest.mark.parametrize("mode", ["f64", "f32_refine"])
def test_equivariances_nside1024_tables(mode):
    """nside 1024, lmax 2048, per-order tables (the benchmark's strategy), 16 maps:
    a CMB-like map of the benchmark recipe and three white-noise maps, each
    with its images."""
    _check(1024, mode, 2, 3, 600)


@pytest.mark.parametrize("mode", ["f64", "f32_refine"])
def test_equivariances_nside2048_staged(mode):
    """nside 2048, lmax 4096, staged strategy (the per-order tables do not fit):
    a CMB-like map of the nside-2048 recipe and a white-noise map with their
    images (8 maps): the analysis sweeps, the staged GEMMs and, in the
    refinement, the synthesis sweeps and the residual fold see every order."""
    _check(2048, mode, 4, 1, 700)
