"""Workgroup schedules of the grouped GEMMs and the autotuner that picks them
(hp2sph_set_schedule, hp2sph_autotune, hp2sph_schedules).

A schedule only decides which workgroup computes which output tile, and each
tile sums its k steps in a fixed order, so every schedule must give the same
a_lm bit for bit.  Before each run the plan's workspace and the output are
cleared, so a schedule that dropped a tile would leave zeros behind and
fail the comparison.  One plan per mode and strategy, with several GEMM
tiles per order (nside 64, 9 maps) and an uneven batch; the FP64 results are
also checked against the oracle."""

import numpy as np
import pytest

import oracle as O
from gpu_util import white_map, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1904_10514_amd as P   # noqa: E402


def _run_clean(plan, maps, iterative):
    plan._ws.zero_()
    out = torch.zeros(plan.alm_total, dtype=torch.complex128, device="cuda")
    if iterative:
        plan.analyze_iterative(maps, 2, out=out)
    else:
        plan.analyze(maps, out=out)
    torch.cuda.synchronize()
    return out.cpu()


CASES = [
    ("f64", "tables", [64] * 9, None),
    ("f64", "staged", [64] * 3, None),
    ("f32_refine", "tables", [64] * 9, None),
    ("f32_refine", "staged", [32] * 2, None),
    ("equal_weight", "tables", [32] * 9, None),
    ("equal_weight", "staged", [32] * 2, None),
    ("f32_refine", "auto", [8, 16, 8, 32, 16, 64, 16, 16, 16, 16, 16, 16, 16, 16], None),
]


@pytest.mark.parametrize("mode,strategy,nsides,lmaxs", CASES)
def test_every_schedule_gives_the_same_result(mode, strategy, nsides, lmaxs):
    maps_np = [white_map(ns, 1700 + i) for i, ns in enumerate(nsides)]
    maps = torch.from_numpy(np.concatenate(maps_np)).cuda()
    plan = P.Plan(nsides, lmaxs, mode=mode, strategy=strategy)
    iterative = mode == "equal_weight"
    # defaults: XCD placement for the per-order GEMMs (thousands of problems),
    # list order with row tiles fastest for the staged ones (four
    # parity-block problems)
    assert plan.schedules
    if strategy == "tables":
        assert all(s == "xcd_round_robin" for s in plan.schedules)
    elif strategy == "staged":
        assert all(s == "linear_rows" for s in plan.schedules)
    results = {}
    for name in P.SCHEDULES:
        plan.set_schedule(name)
        results[name] = _run_clean(plan, maps, iterative)
    ref = results["xcd_round_robin"]
    for name, r in results.items():
        print(f"{mode} {strategy} {name}: equal={torch.equal(r, ref)}")
        assert torch.equal(r, ref), name
    if mode == "f64" and len(set(nsides)) == 1:
        oracle = np.concatenate([O.analyze(f, nsides[0]) for f in maps_np])
        assert rel_err(ref.numpy(), oracle) < 1e-12
    plan.close()


@pytest.mark.parametrize("mode", ["f32_refine", "equal_weight"])
def test_autotune_keeps_the_result_and_reports_its_choice(mode):
    nsides = [64] * 9
    maps = torch.from_numpy(np.concatenate([white_map(ns, 1800 + i) for i, ns in enumerate(nsides)])).cuda()
    plan = P.Plan(nsides, mode=mode, strategy="tables")
    before = _run_clean(plan, maps, False)
    ms, alm = plan.autotune(maps, reps=2)
    torch.cuda.synchronize()
    chosen = plan.schedules
    print(f"{mode}: {ms:.3f} ms per analysis, schedules {chosen}")
    assert ms > 0.0
    assert len(chosen) == (3 if mode == "f32_refine" else 2)
    assert all(c in P.SCHEDULES for c in chosen)
    assert torch.equal(alm.cpu(), before)             # autotune leaves alm = analyze(maps)
    assert torch.equal(_run_clean(plan, maps, False), before)
    plan.close()


def test_autotune_pauses_stage_profiling():
    nside = 32
    maps = torch.from_numpy(white_map(nside, 1900)).cuda()
    plan = P.Plan(nside, batch=1, mode="f64")
    plan.profile(True)
    plan.analyze(maps)
    plan.autotune(maps, reps=1)
    prof = plan.profile_read()
    assert prof["gemm_analysis"][1] == 1               # only the analysis before autotune
    plan.analyze(maps)
    assert plan.profile_read()["gemm_analysis"][1] == 2  # recording resumed
    plan.profile(False)
    plan.close()


def test_schedule_and_autotune_argument_errors():
    nside = 16
    maps = torch.from_numpy(white_map(nside, 1950)).cuda()
    plan = P.Plan(nside, batch=1, mode="f64")
    with pytest.raises(ValueError):
        plan.set_schedule("nonexistent")
    lib = P.lib()
    assert lib.hp2sph_set_schedule(plan._h, P.HP2SPH_F64 - 1) == -1          # EINVAL
    assert lib.hp2sph_set_schedule(plan._h, len(P.SCHEDULES)) == -1
    with pytest.raises(P.HP2SPHError):
        plan.autotune(maps, reps=0)
    with pytest.raises(P.HP2SPHError):
        plan.autotune(maps, reps=P.MAX_TUNE_REPS + 1)
    plan.close()


@pytest.mark.parametrize("mode", ["f32_refine", "f64"])
def test_work_lists_over_mixed_groups(mode):
    """Every stage runs as one work list over all nside groups.  The batch
    mixes per-order-table groups (>= 8 maps) and staged ones; the fold's
    persistent grids only change which workgroup takes which item (items keep
    their XCD), the pack's tile shapes only which workgroup moves which
    a_lm and the ring orders only which workgroup transforms which ring pair,
    so every option gives the same a_lm bit for bit; 512 ring-transform
    threads (radix-8 passes) change the FFT's rounding only; and each map
    agrees with its own single-map analysis (bitwise for the staged groups,
    whose single-map plans run the same strategy) and with the oracle."""
    nsides = [32] * 9 + [16, 8, 16] + [64] * 8 + [4]
    maps_np = [white_map(ns, 1900 + i) for i, ns in enumerate(nsides)]
    maps = torch.from_numpy(np.concatenate(maps_np)).cuda()
    plan = P.Plan(nsides, mode=mode)
    assert plan.option("fold_grid") == 0 and plan.option("pack_maps") == 32 and plan.option("ring_order") == 0
    assert plan.option("ring_threads") == 256
    ref = _run_clean(plan, maps, False)
    for name, value in [("fold_grid", 8), ("fold_grid", 64), ("fold_grid", 256), ("fold_grid", 2048),
                        ("pack_maps", 16), ("pack_maps", 64), ("fold_grid", 0), ("ring_order", 1),
                        ("ring_order", 2)]:
        plan.set_option(name, value)
        assert plan.option(name) == value
        got = _run_clean(plan, maps, False)
        print(f"{mode} {name} {value}: equal={torch.equal(got, ref)}")
        assert torch.equal(got, ref), (name, value)
    plan.set_option("ring_threads", 512)
    got = _run_clean(plan, maps, False)
    diff = rel_err(got.numpy(), ref.numpy())
    print(f"{mode} ring_threads 512: rel diff {diff:.3e}")
    assert diff < (1e-13 if mode == "f64" else 1e-6)
    plan.set_option("ring_threads", 256)
    assert torch.equal(_run_clean(plan, maps, False), ref)
    for name, value in [("fold_grid", 3), ("fold_grid", -8), ("pack_maps", 8), ("pack_maps", 48), ("ring_order", 3),
                        ("ring_threads", 128), ("ring_threads", 1024)]:
        with pytest.raises(P.HP2SPHError):
            plan.set_option(name, value)
    with pytest.raises(ValueError):
        plan.set_option("tiles", 1)
    ref = ref.numpy()
    offs = plan.alm_offsets
    plan.close()
    for i, ns in enumerate(nsides):
        single = P.Plan(ns, mode=mode)
        a = single.analyze(torch.from_numpy(maps_np[i]).cuda()).cpu().numpy()
        single.close()
        mine = ref[offs[i]:offs[i + 1]]
        if nsides.count(ns) < 8:
            assert np.array_equal(mine, a), i
        if mode == "f64":
            assert rel_err(mine, O.analyze(maps_np[i], ns)) < 1e-12
        else:
            assert rel_err(mine, O.analyze_refined(maps_np[i], ns)) < 1e-6
