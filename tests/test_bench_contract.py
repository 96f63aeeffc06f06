"""CPU checks of bench.py's contract: one GPU only, and every stage it times
has a positive algorithmic work figure for its roofline fraction."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


STAGES = {
    "f32_refine": ["ring_forward", "gemm_analysis", "pack", "unpack", "gemm_synthesis", "cl", "residual_fold"],
    "f64": ["ring_forward", "gemm_analysis", "pack", "cl"],
    "equal_weight": ["ring_adjoint", "gemm_adjoint", "gemm_synthesis", "residual_fold", "unpack", "pack"],
}


@pytest.mark.parametrize("mode", sorted(STAGES))
@pytest.mark.parametrize("strategy", ["tables", "staged"])
def test_every_timed_stage_has_work(mode, strategy):
    for st in STAGES[mode]:
        dt = bench.stage_dtype(st, mode)
        kind, amount = bench.stage_work(st, 1024, 64, 4 if dt == "f32" else 8, strategy, mode)
        assert amount > 0, (mode, strategy, st)
        assert kind == ("flop" if st.startswith("gemm") else "byte")
        assert bench.stage_bound(st) == ("mfma" if st.startswith("gemm") else "hbm")


def test_per_order_gemm_flops_count_every_coefficient_once():
    """Counted over (l, m) instead of the four parity blocks: every a_l^m with
    0 <= m <= l <= p is one row of one order's table, contracted over the ring
    rows it uses (synthesis: 2 nside; analysis: the rows h >= ceil(m/2) of
    the 2 nside + 1, all for m = 0) with 2 flops per term and 2B columns."""
    for nside, B in ((8, 3), (64, 5), (1024, 64)):
        p = 2 * nside
        syn = (p + 1) * (p + 2) // 2 * (2 * nside) * 2 * (2 * B)
        ana = sum((p - m + 1) * (2 * nside + 1 - (0 if m == 0 else (m + 1) // 2)) for m in range(p + 1)) * 2 * (2 * B)
        assert bench.order_gemm_flops(nside, B, True) == syn
        assert bench.order_gemm_flops(nside, B, False) == ana


def test_measured_traffic_is_per_launch():
    """The committed counter summaries hold per-dispatch means (FETCH_SIZE and
    WRITE_SIZE in KiB, averaged over the dispatches used, then scaled); the
    bench's roofline traffic is that mean, not divided again."""
    import glob
    import json
    paths = sorted(glob.glob(os.path.join(ROOT, "profiles", "hbm_traffic_*.json")))
    assert paths
    for path in paths:
        js = json.load(open(path))
        wl = js["workload"]
        for key, e in js["stages"].items():
            stage, dt = key.split("/")
            got = bench.measured_traffic(stage, dt, wl["nside"], wl["batch"], wl["strategy"])
            if got is None:   # kernels changed since the counters were taken
                pytest.skip("counter summary is older than the kernels")
            assert got == pytest.approx(1024 * (e["fetch_kib"] * js["calibration"]["fetch_scale"] +
                                                e["write_kib"] * js["calibration"]["write_scale"]), rel=1e-12)
    # a workload without counter runs, or another strategy, has no measured traffic
    assert bench.measured_traffic("gemm_synthesis", "f64", 512, 3, "tables") is None
    assert bench.measured_traffic("gemm_synthesis", "f64", 1024, 64, "staged") is None
