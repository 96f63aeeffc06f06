"""The allocation-free analysis, hp2sph_analyze_noalloc (the library's static
device workspace instead of a caller's), through the C ABI against
hp2sph_analyze on the same plan and maps: two calls in a row, the second with
a smaller input, each bitwise equal to the workspace entry point (both run the
same kernels in the same order), nothing allocated by the call, and a plan
whose workspace exceeds the static one refused before any launch."""

import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1904_10514_amd as P   # noqa: E402
from gpu_util import white_map      # noqa: E402

EINVAL = -1


def _noalloc_vs_workspace(nside, nmaps, mode, strategy, seed):
    lib = P.lib()
    maps = np.concatenate([white_map(nside, seed + v) for v in range(nmaps)])
    dev = torch.from_numpy(maps).cuda()
    plan = P.Plan(nside, batch=nmaps, mode=mode, strategy=strategy)
    assert plan.strategy == strategy
    assert plan.workspace_bytes <= P.NOALLOC_WORKSPACE
    ref = plan.analyze(dev)
    out = torch.full_like(ref, float("nan"))
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.hp2sph_analyze_noalloc(plan._h, dev.data_ptr(), out.data_ptr(), stream)
    assert rc == 0, lib.hp2sph_last_error()
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0          # the call allocated nothing
    ok = torch.equal(out, ref)
    plan.close()
    return ok


def test_noalloc_matches_the_workspace_entry_point_on_two_calls():
    # first call: the larger input (FP32 + refinement, per-order tables, 8 maps
    # of nside 64); second: a smaller one (FP64, staged, 2 maps of nside 16),
    # which runs on the static workspace the first call left behind
    assert _noalloc_vs_workspace(64, 8, "f32_refine", "tables", 2400)
    assert _noalloc_vs_workspace(16, 2, "f64", "staged", 2500)


def test_noalloc_refuses_a_plan_larger_than_the_static_workspace():
    lib = P.lib()
    nside, nmaps = 512, 8
    plan = P.Plan(nside, batch=nmaps, mode="f64", strategy="staged")
    assert plan.workspace_bytes > P.NOALLOC_WORKSPACE
    maps = torch.zeros(plan.npix_total, dtype=torch.float64, device="cuda")
    out = torch.zeros(plan.alm_total, dtype=torch.complex128, device="cuda")
    assert lib.hp2sph_analyze_noalloc(plan._h, maps.data_ptr(), out.data_ptr(), None) == EINVAL
    assert b"static workspace" in lib.hp2sph_last_error()
    torch.cuda.synchronize()
    plan.close()
