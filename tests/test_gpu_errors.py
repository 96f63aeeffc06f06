"""Error paths of the C ABI that need a plan (and so a GPU): every call below
must fail with the documented code before it launches anything."""

import ctypes

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1904_10514_amd as P   # noqa: E402

EINVAL, ENOMEM, EWORKSPACE, ESTATE = -1, -2, -4, -5


def test_misaligned_pointers_and_workspace_are_rejected():
    lib = P.lib()
    plan = P.Plan(8, mode="f64")
    maps = torch.zeros(P.npix(8) + 1, dtype=torch.float64, device="cuda")
    alm = torch.zeros(2 * P.alm_size(16) + 2, dtype=torch.float64, device="cuda")
    h, ws, nb = plan._h, plan._ws_ptr, plan.workspace_bytes
    # maps and alm must be 16-byte aligned
    assert lib.hp2sph_analyze(h, maps.data_ptr() + 8, alm.data_ptr(), ws, nb, None) == EINVAL
    assert lib.hp2sph_analyze(h, maps.data_ptr(), alm.data_ptr() + 8, ws, nb, None) == EINVAL
    assert lib.hp2sph_analyze(h, None, alm.data_ptr(), ws, nb, None) == EINVAL
    # the workspace must be given, 256-byte aligned and large enough
    assert lib.hp2sph_analyze(h, maps.data_ptr(), alm.data_ptr(), None, nb, None) == EWORKSPACE
    assert lib.hp2sph_analyze(h, maps.data_ptr(), alm.data_ptr(), ws + 128, nb, None) == EWORKSPACE
    assert b"workspace" in lib.hp2sph_last_error()
    assert lib.hp2sph_analyze(h, maps.data_ptr(), alm.data_ptr(), ws, nb - 1, None) == EWORKSPACE
    assert b"smaller" in lib.hp2sph_last_error()
    assert lib.hp2sph_synthesize(h, alm.data_ptr(), maps.data_ptr(), ws, nb - 256, None) == EWORKSPACE
    torch.cuda.synchronize()
    plan.close()


def test_iteration_count_is_checked():
    lib = P.lib()
    plan = P.Plan(8, mode="equal_weight")
    maps = torch.zeros(P.npix(8), dtype=torch.float64, device="cuda")
    alm = torch.zeros(2 * P.alm_size(16), dtype=torch.float64, device="cuda")
    nb = plan.workspace_bytes
    assert lib.hp2sph_analyze_iterative(plan._h, maps.data_ptr(), alm.data_ptr(), -1, plan._ws_ptr, nb, None) == EINVAL
    assert b"niter" in lib.hp2sph_last_error()
    assert lib.hp2sph_analyze_iterative(plan._h, maps.data_ptr(), alm.data_ptr(), 0, plan._ws_ptr, nb - 8,
                                        None) == EWORKSPACE
    assert lib.hp2sph_analyze_iterative(plan._h, maps.data_ptr(), alm.data_ptr(), 0, plan._ws_ptr, nb, None) == 0
    torch.cuda.synchronize()
    plan.close()


def test_destroyed_plan_is_refused_without_being_read():
    lib = P.lib()
    plan = P.Plan(8, mode="f64")
    h = plan._h
    assert lib.hp2sph_plan_destroy(h) == 0
    assert lib.hp2sph_plan_destroy(h) == ESTATE          # a second destroy is reported
    ws = ctypes.c_size_t()
    assert lib.hp2sph_workspace_size(h, ctypes.byref(ws)) == ESTATE
    plan._h = None


def test_binding_checks_every_buffer_before_a_launch():
    """The C ABI takes raw pointers: wrong dtypes, sizes, layouts or devices of
    inputs and out= buffers are refused by the binding before any call."""
    nside, lmax = 8, 16
    plan = P.Plan(nside, lmax, mode="f64")
    maps = torch.zeros(P.npix(nside), dtype=torch.float64, device="cuda")
    alm = plan.analyze(maps)
    good_cl = torch.empty(lmax + 1, dtype=torch.float64, device="cuda")
    bad = [
        lambda: plan.analyze(maps, out=torch.empty(P.alm_size(lmax) - 1, dtype=torch.complex128, device="cuda")),
        lambda: plan.analyze(maps, out=torch.empty(P.alm_size(lmax), dtype=torch.complex64, device="cuda")),
        lambda: plan.analyze(maps, out=torch.empty(2 * P.alm_size(lmax), dtype=torch.complex128, device="cuda")[::2]),
        lambda: plan.analyze(maps, out=torch.empty(P.alm_size(lmax), dtype=torch.complex128)),
        lambda: plan.analyze(maps.float()),
        lambda: plan.analyze(maps[:-1]),
        lambda: plan.power_spectrum(alm[:-1]),
        lambda: plan.power_spectrum(alm.to(torch.complex64)),
        lambda: plan.power_spectrum(alm, out=good_cl[:-1]),
        lambda: plan.power_spectrum(alm, out=good_cl.float()),
        lambda: plan.synthesize(alm, out=maps[:-1]),
        lambda: plan.synthesize(alm.view(torch.float64)),
        lambda: plan.autotune(maps, out=alm[:-1]),
    ]
    for i, call in enumerate(bad):
        with pytest.raises(ValueError):
            call()
    plan.power_spectrum(alm, out=good_cl)
    torch.cuda.synchronize()
    plan.close()


def test_oversized_tables_give_enomem_and_leak_nothing():
    """Per-order tables of an FP32+refinement plan at nside 2048 (about 390 GB)
    cannot fit: plan creation refuses them before building anything, and the
    free device memory is unchanged afterwards; so is it after a plan that
    fits is created and destroyed."""
    import gc
    lib = P.lib()
    h = ctypes.c_void_p()
    ns = (ctypes.c_int32 * 8)(*([64] * 8))
    lm = (ctypes.c_int32 * 8)(*([128] * 8))
    # one plan built and freed first, so that run-time pools the HIP runtime
    # keeps for the process (kernel arguments, code objects) exist already
    assert lib.hp2sph_plan_create_ex(ns, lm, 8, P.HP2SPH_F32_REFINE, P.STRATEGIES["tables"], ctypes.byref(h)) == 0
    assert lib.hp2sph_plan_destroy(h) == 0
    gc.collect()
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    ns = (ctypes.c_int32 * 16)(*([2048] * 16))
    lm = (ctypes.c_int32 * 16)(*([4096] * 16))
    assert lib.hp2sph_plan_create_ex(ns, lm, 16, P.HP2SPH_F32_REFINE, P.STRATEGIES["tables"], ctypes.byref(h)) == ENOMEM
    assert b"tables" in lib.hp2sph_last_error()
    assert not h.value
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0
    ns = (ctypes.c_int32 * 8)(*([64] * 8))
    lm = (ctypes.c_int32 * 8)(*([128] * 8))
    assert lib.hp2sph_plan_create_ex(ns, lm, 8, P.HP2SPH_F32_REFINE, P.STRATEGIES["tables"], ctypes.byref(h)) == 0
    assert torch.cuda.mem_get_info()[0] < free0
    assert lib.hp2sph_plan_destroy(h) == 0
    gc.collect()
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
