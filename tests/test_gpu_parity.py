"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle."""

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import cmb_map, white_map, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1904_10514_amd as P   # noqa: E402

# FP64 parity bar: max |a_gpu - a_oracle| <= TOL64 * max |a|, and the same
# relative bar per C_l.  The two sides differ only in rounding order
# (FFT vs direct sums, QR-built tables vs QR lstsq, sweeps vs quadrature);
# 1e-12 leaves ~100x headroom over the measured ~1e-14.
TOL64 = 1e-12
# FP32 + one FP64 refinement round vs the same recipe in FP64: the round
# leaves the FP32 error of the first pass (eps32 = 6e-8 times the growth of the
# p-term sums, measured 1.5-2.2e-7 for one pass) times I - A S, the method's own
# error on the residual, whose norm reaches ~1 on white noise at small nside
# (polar rings alias most modes), plus the FP32 error of the correction: 1e-6.
# (Smooth maps land at 4e-10 - 1.5e-8.)  That the residual itself is formed in
# FP64 is checked at full size on exactly recovered fields
# (tests/test_gpu_fullsize.py), where the refined error must fall to 1e-10.
TOL_REFINE = 1e-6


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _gpu_analyze(maps, nside, lmax=None, mode="f64"):
    plan = P.Plan(nside, lmax, mode=mode)
    a = plan.analyze(_dev(maps))
    cl = plan.power_spectrum(a)
    torch.cuda.synchronize()
    return a.cpu().numpy(), cl.cpu().numpy()


@pytest.mark.parametrize("nside", [2, 4, 8, 16, 64])
def test_f64_analysis_white_noise(nside):
    f = white_map(nside, nside)
    a, cl = _gpu_analyze(f, nside)
    ref = O.analyze(f, nside)
    print(f"nside {nside}: rel err {rel_err(a, ref):.3e}")
    assert rel_err(a, ref) < TOL64
    clr = O.power_spectrum(ref, 2 * nside)
    assert np.max(np.abs(cl - clr) / clr) < TOL64


def test_f64_analysis_config_nside16_L32():
    """The one-map nside 16 / lmax 32 workload, C_l = 1/(l(l+1))."""
    f, _ = cmb_map(0, 0, 16, 32)
    a, cl = _gpu_analyze(f, 16, 32)
    ref = O.analyze(f, 16, 32)
    assert rel_err(a, ref) < TOL64
    clr = O.power_spectrum(ref, 32)
    assert np.max(np.abs(cl[2:] - clr[2:]) / clr[2:]) < TOL64


@pytest.mark.parametrize("nside,lmax", [(8, 5), (16, 20), (32, 0)])
def test_f64_lmax_truncation(nside, lmax):
    f = white_map(nside, 100 + nside)
    a, _ = _gpu_analyze(f, nside, lmax)
    ref = O.analyze(f, nside, lmax)
    assert a.shape[0] == O.alm_size(lmax)
    assert rel_err(a, ref) < TOL64


def test_constant_map_on_gpu():
    nside = 32
    a, cl = _gpu_analyze(np.full(O.npix(nside), 1.25), nside)
    assert a[0] == pytest.approx(np.sqrt(4 * np.pi) * 1.25, rel=1e-14)
    assert np.max(np.abs(a[1:])) < 1e-13


@pytest.mark.parametrize("nside", [2, 8, 32])
def test_synthesis_vs_oracle(nside):
    lmax = 2 * nside
    rng = np.random.default_rng(5)
    a = rng.standard_normal(O.alm_size(lmax)) + 1j * rng.standard_normal(O.alm_size(lmax))
    for l in range(lmax + 1):
        a[O.alm_index(l, 0, lmax)] = a[O.alm_index(l, 0, lmax)].real
    plan = P.Plan(nside, lmax, mode="f64")
    f = plan.synthesize(_dev(a)).cpu().numpy()
    ref = O.synthesize(a, nside, lmax)
    assert rel_err(f, ref) < TOL64


def test_uneven_batch_equals_single_maps():
    nsides = [8, 16, 8, 4, 16]
    maps = [white_map(n, 200 + i) for i, n in enumerate(nsides)]
    plan = P.Plan(nsides, mode="f64")
    a = plan.analyze(_dev(np.concatenate(maps))).cpu().numpy()
    for i, n in enumerate(nsides):
        ai = a[plan.alm_offsets[i]:plan.alm_offsets[i + 1]]
        assert rel_err(ai, O.analyze(maps[i], n)) < TOL64
        single, _ = _gpu_analyze(maps[i], n)
        assert np.array_equal(ai, single)


def test_batch_members_are_independent():
    nside = 16
    maps = [white_map(nside, 300 + i) for i in range(3)]
    plan = P.Plan(nside, batch=3, mode="f64")
    a = plan.analyze(_dev(np.concatenate(maps))).cpu().numpy()
    sz = O.alm_size(2 * nside)
    for i in range(3):
        single, _ = _gpu_analyze(maps[i], nside)
        assert np.array_equal(a[i * sz:(i + 1) * sz], single)


def test_f64_analysis_nside256_L512():
    """The one-map nside 256 / lmax 512 workload with a beamed power-law spectrum."""
    f, _ = cmb_map(1, 0, 256, 512)
    a, cl = _gpu_analyze(f, 256, 512)
    ref = O.analyze(f, 256, 512)
    print(f"nside 256: rel err {rel_err(a, ref):.3e}")
    assert rel_err(a, ref) < TOL64


@pytest.mark.parametrize("nside", [8, 32, 64])
def test_f32_refine_vs_refined_oracle(nside):
    """FP32 stages + one FP64-residual round against the same recipe in FP64."""
    f, _ = cmb_map(1, nside, nside)
    plan = P.Plan(nside, mode="f32_refine")
    a = plan.analyze(_dev(f))
    cl = plan.power_spectrum(a)
    torch.cuda.synchronize()
    a, cl = a.cpu().numpy(), cl.cpu().numpy()
    ref = O.analyze_refined(f, nside)
    plain = O.analyze(f, nside)
    clr = O.power_spectrum(ref, 2 * nside)
    e_ref = rel_err(a, ref)
    e_plain = rel_err(a, plain)
    e_cl = float(np.max(np.abs(cl[2:] - clr[2:]) / clr[2:]))
    print(f"nside {nside}: vs O_ref {e_ref:.3e}, vs O_plain {e_plain:.3e}, rel C_l {e_cl:.3e}")
    assert e_ref < TOL_REFINE


@pytest.mark.parametrize("nside", [16, 64])
def test_f32_single_pass_vs_oracle(nside):
    f, _ = cmb_map(1, 100 + nside, nside)
    plan = P.Plan(nside, mode="f32")
    a = plan.analyze(_dev(f)).cpu().numpy()
    e = rel_err(a, O.analyze(f, nside))
    print(f"nside {nside}: f32 single pass rel err {e:.3e}")
    assert e < 1e-5


# ---- per-order tables strategy (sweeps applied at plan creation) ----

@pytest.mark.parametrize("nside,nb", [(2, 1), (4, 3), (16, 2), (64, 2)])
def test_tables_f64_vs_oracle(nside, nb):
    maps = [white_map(nside, 400 + nside + i) for i in range(nb)]
    plan = P.Plan(nside, batch=nb, mode="f64", strategy="tables")
    assert plan.strategy == "tables"
    a = plan.analyze(_dev(np.concatenate(maps))).cpu().numpy()
    sz = O.alm_size(2 * nside)
    for i in range(nb):
        e = rel_err(a[i * sz:(i + 1) * sz], O.analyze(maps[i], nside))
        print(f"tables nside {nside} map {i}: rel err {e:.3e}")
        assert e < TOL64


def test_tables_and_staged_agree_on_uneven_batch():
    nsides = [16, 8, 16, 32, 8]
    maps = np.concatenate([white_map(n, 500 + i) for i, n in enumerate(nsides)])
    lmax = [2 * n - (i % 2) for i, n in enumerate(nsides)]
    a_t = P.Plan(nsides, lmax, mode="f64", strategy="tables").analyze(_dev(maps)).cpu().numpy()
    a_s = P.Plan(nsides, lmax, mode="f64", strategy="staged").analyze(_dev(maps)).cpu().numpy()
    assert rel_err(a_t, a_s) < TOL64


@pytest.mark.parametrize("nside", [8, 32])
def test_tables_f32_refine_vs_refined_oracle(nside):
    f, _ = cmb_map(1, 600 + nside, nside)
    plan = P.Plan(nside, batch=1, mode="f32_refine", strategy="tables")
    assert plan.strategy == "tables"
    a = plan.analyze(_dev(f)).cpu().numpy()
    e = rel_err(a, O.analyze_refined(f, nside))
    print(f"tables f32+refine nside {nside}: vs O_ref {e:.3e}")
    assert e < TOL_REFINE


def test_tables_synthesis_path_in_refinement_matches_staged():
    """The FP64 synthesis of the refinement through the tables equals the staged one."""
    nside = 16
    rng = np.random.default_rng(7)
    lmax = 2 * nside
    a = rng.standard_normal(O.alm_size(lmax)) + 1j * rng.standard_normal(O.alm_size(lmax))
    for l in range(lmax + 1):
        a[O.alm_index(l, 0, lmax)] = a[O.alm_index(l, 0, lmax)].real
    pt = P.Plan(nside, batch=1, mode="f32_refine", strategy="tables")
    f = pt.synthesize(_dev(a)).cpu().numpy()
    assert rel_err(f, O.synthesize(a, nside, lmax)) < TOL64


def test_tables_f64_plan_synthesis_uses_staged_path_correctly():
    """An F64 tables plan synthesises through the staged sweeps (map-major)."""
    nside, nb = 8, 3
    lmax = 2 * nside
    rng = np.random.default_rng(8)
    a = rng.standard_normal(nb * O.alm_size(lmax)) + 1j * rng.standard_normal(nb * O.alm_size(lmax))
    for i in range(nb):
        for l in range(lmax + 1):
            k = i * O.alm_size(lmax) + O.alm_index(l, 0, lmax)
            a[k] = a[k].real
    plan = P.Plan(nside, batch=nb, mode="f64", strategy="tables")
    f = plan.synthesize(_dev(a)).cpu().numpy()
    sz, npx = O.alm_size(lmax), O.npix(nside)
    for i in range(nb):
        ref = O.synthesize(a[i * sz:(i + 1) * sz], nside, lmax)
        assert rel_err(f[i * npx:(i + 1) * npx], ref) < TOL64


@pytest.mark.parametrize("strategy", ["staged", "tables"])
def test_f32_refine_truncated_lmax_vs_refined_oracle(strategy):
    """lmax < p: the refinement synthesises a0 truncated at lmax (reading R15)."""
    nside, lmax = 16, 25
    f, _ = cmb_map(1, 700, nside)
    plan = P.Plan(nside, lmax, batch=1, mode="f32_refine", strategy=strategy)
    a = plan.analyze(_dev(f)).cpu().numpy()
    e = rel_err(a, O.analyze_refined(f, nside, lmax))
    print(f"f32+refine nside {nside} lmax {lmax} ({strategy}): vs O_ref {e:.3e}")
    assert e < TOL_REFINE


def test_f32_refine_uneven_batch_vs_refined_oracle():
    """Uneven nside and lmax in one refinement plan, each map against O_ref."""
    nsides = [8, 16, 8, 32]
    lmaxs = [16, 30, 13, 64]
    maps = [white_map(n, 800 + i) for i, n in enumerate(nsides)]
    plan = P.Plan(nsides, lmaxs, mode="f32_refine")
    a = plan.analyze(_dev(np.concatenate(maps))).cpu().numpy()
    off = 0
    for f, n, L in zip(maps, nsides, lmaxs):
        sz = O.alm_size(L)
        e = rel_err(a[off:off + sz], O.analyze_refined(f, n, L))
        print(f"uneven f32+refine nside {n} lmax {L}: vs O_ref {e:.3e}")
        assert e < TOL_REFINE
        off += sz


@pytest.mark.parametrize("strategy", ["staged", "tables"])
@pytest.mark.parametrize("mode", ["f64", "f32_refine"])
def test_several_tiles_nside128(mode, strategy):
    """nside 128, 3 maps: the per-order analysis tables have up to 129 rows
    (a second 128-row tile holding one row), 257 - ceil(m/2) ring rows (ragged
    k steps) and 6 columns per order; the synthesis tables of the refinement
    span two full tiles."""
    nside, batch = 128, 3
    maps = [white_map(nside, 1300 + v) for v in range(batch)]
    plan = P.Plan(nside, batch=batch, mode=mode, strategy=strategy)
    a = plan.analyze(_dev(np.concatenate(maps)))
    torch.cuda.synchronize()
    a = a.cpu().numpy()
    plan.close()
    route = O.analyze if mode == "f64" else O.analyze_refined
    ref = np.concatenate([route(f, nside) for f in maps])
    err = rel_err(a, ref)
    print(f"{mode} {strategy} nside 128 x 3: {err:.3e}")
    assert err < (TOL64 if mode == "f64" else TOL_REFINE)


@pytest.mark.parametrize("mode", ["f64", "f32_refine"])
def test_batch_widths_match_single_maps_bitwise(mode):
    """Per-order GEMMs of 2 B columns: B = 9, 20, 40, 73 maps leave 18, 40,
    80 (one full and one partial 64-column wave half) and 146 columns (a
    second column tile with 18 live columns), so every count of live
    16-column blocks per wave is met.  Each column of a GEMM is computed
    alone, so every map of the batch must equal its single-map analysis bit
    for bit (and the single maps agree with the oracle)."""
    nside = 8
    route = O.analyze if mode == "f64" else O.analyze_refined
    maps = [white_map(nside, 1500 + v) for v in range(73)]
    singles = []
    for v in range(73):
        plan = P.Plan(nside, batch=1, mode=mode, strategy="tables")
        singles.append(plan.analyze(_dev(maps[v])).cpu().numpy())
        plan.close()
    for v in (0, 40, 72):
        assert rel_err(singles[v], route(maps[v], nside)) < (TOL64 if mode == "f64" else TOL_REFINE)
    sz = O.alm_size(2 * nside)
    for batch in (9, 20, 40, 73):
        plan = P.Plan(nside, batch=batch, mode=mode, strategy="tables")
        a = plan.analyze(_dev(np.concatenate(maps[:batch]))).cpu().numpy()
        plan.close()
        for v in range(batch):
            assert np.array_equal(a[v * sz:(v + 1) * sz], singles[v]), (batch, v)


@pytest.mark.parametrize("mode", ["f64", "f32_refine"])
def test_staged_sweep_map_groups_match_single_maps_bitwise(mode):
    """Staged plans of 1, 2, 3, 5 and 7 maps: the Givens sweeps carry one
    map per lane for a single map and two otherwise (a partial last map
    group for odd batches), and
    each map's rotations keep their own fma order, so every map of a batch
    equals its single-map analysis bit for bit; the single maps agree with
    the oracle."""
    nside = 16
    route = O.analyze if mode == "f64" else O.analyze_refined
    maps = [white_map(nside, 1600 + v) for v in range(7)]
    singles = []
    for v in range(7):
        plan = P.Plan(nside, batch=1, mode=mode, strategy="staged")
        singles.append(plan.analyze(_dev(maps[v])).cpu().numpy())
        plan.close()
    for v in (0, 6):
        assert rel_err(singles[v], route(maps[v], nside)) < (TOL64 if mode == "f64" else TOL_REFINE)
    sz = O.alm_size(2 * nside)
    for batch in (2, 3, 5, 7):
        plan = P.Plan(nside, batch=batch, mode=mode, strategy="staged")
        a = plan.analyze(_dev(np.concatenate(maps[:batch]))).cpu().numpy()
        plan.close()
        for v in range(batch):
            assert np.array_equal(a[v * sz:(v + 1) * sz], singles[v]), (batch, v)
