"""Error paths of the C ABI that need a plan (and so a GPU): every call below
must fail with the documented code before it launches anything."""

import ctypes

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1904_10514_amd as P   # noqa: E402

EINVAL, EWORKSPACE = -1, -4


def test_misaligned_pointers_and_workspace_are_rejected():
    lib = P.lib()
    plan = P.Plan(8, mode="f64")
    maps = torch.zeros(P.npix(8) + 1, dtype=torch.float64, device="cuda")
    alm = torch.zeros(2 * P.alm_size(16) + 2, dtype=torch.float64, device="cuda")
    h, ws = plan._h, plan._ws_ptr
    # maps and alm must be 16-byte aligned
    assert lib.hp2sph_analyze(h, maps.data_ptr() + 8, alm.data_ptr(), ws, None) == EINVAL
    assert lib.hp2sph_analyze(h, maps.data_ptr(), alm.data_ptr() + 8, ws, None) == EINVAL
    assert lib.hp2sph_analyze(h, None, alm.data_ptr(), ws, None) == EINVAL
    # the workspace must be given and 256-byte aligned
    assert lib.hp2sph_analyze(h, maps.data_ptr(), alm.data_ptr(), None, None) == EWORKSPACE
    assert lib.hp2sph_analyze(h, maps.data_ptr(), alm.data_ptr(), ws + 128, None) == EWORKSPACE
    assert b"workspace" in lib.hp2sph_last_error()
    torch.cuda.synchronize()
    plan.close()


def test_iteration_count_is_checked():
    lib = P.lib()
    plan = P.Plan(8, mode="equal_weight")
    maps = torch.zeros(P.npix(8), dtype=torch.float64, device="cuda")
    alm = torch.zeros(2 * P.alm_size(16), dtype=torch.float64, device="cuda")
    assert lib.hp2sph_analyze_iterative(plan._h, maps.data_ptr(), alm.data_ptr(), -1, plan._ws_ptr, None) == EINVAL
    assert b"niter" in lib.hp2sph_last_error()
    assert lib.hp2sph_analyze_iterative(plan._h, maps.data_ptr(), alm.data_ptr(), 0, plan._ws_ptr, None) == 0
    torch.cuda.synchronize()
    plan.close()
