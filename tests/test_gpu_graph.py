"""A whole analysis of an uneven batch as one graph launch: the C ABI's
analyze calls only enqueue kernels on the caller's stream (no allocation, no
memset, no synchronisation), so a HIP graph captured around them replays the
batch.  Each replay, with eager work and synchronisations between replays,
must equal the eager result bitwise (every kernel is deterministic: fixed
reduction orders, no atomics)."""

import numpy as np
import pytest

from gpu_util import white_map

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1904_10514_amd as P   # noqa: E402

NSIDES = [8, 16, 8, 32, 16, 64, 8, 16, 16, 16, 16, 16, 16, 16]
LMAXS = [16, 30, 13, 64, 32, 128, 16, 32, 32, 32, 32, 32, 32, 25]


def _capture_and_replay(plan, run, maps, n_replays=4):
    eager = run(maps).clone()
    torch.cuda.synchronize()
    out = torch.empty_like(eager)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run(maps, out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run(maps, out)
    for _ in range(n_replays):
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager)
        again = run(maps)            # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(again, eager)
    return eager


@pytest.mark.parametrize("strategy", ["auto", "tables"])
def test_refined_analysis_of_an_uneven_batch_replays_from_a_graph(strategy):
    maps = torch.from_numpy(np.concatenate([white_map(ns, 900 + i) for i, ns in enumerate(NSIDES)])).cuda()
    plan = P.Plan(NSIDES, LMAXS, mode="f32_refine", strategy=strategy)

    def run(x, out=None):
        return plan.analyze(x, out=out)

    _capture_and_replay(plan, run, maps)
    plan.close()


def test_jacobi_analysis_replays_from_a_graph():
    maps = torch.from_numpy(np.concatenate([white_map(ns, 950 + i) for i, ns in enumerate(NSIDES)])).cuda()
    plan = P.Plan(NSIDES, LMAXS, mode="equal_weight", strategy="tables")

    def run(x, out=None):
        return plan.analyze_iterative(x, 3, out=out)

    _capture_and_replay(plan, run, maps)
    plan.close()
