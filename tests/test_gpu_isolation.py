"""Maps of a batch are independent: a NaN in one map leaves every other map's
a_lm and C_l bitwise unchanged, in both precision modes and both strategies
(the grouped GEMMs mix maps only across output columns, never within one)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1904_10514_amd as P   # noqa: E402
from gpu_util import white_map      # noqa: E402

NSIDE, BATCH, BAD = 32, 8, 3


@pytest.mark.parametrize("strategy", ["staged", "tables"])
@pytest.mark.parametrize("mode", ["f64", "f32_refine"])
def test_nan_in_one_map_stays_in_that_map(mode, strategy):
    maps = np.stack([white_map(NSIDE, 2100 + v) for v in range(BATCH)])
    clean = torch.from_numpy(maps.reshape(-1)).cuda()
    dirty = clean.clone().view(BATCH, -1)
    dirty[BAD, 1234] = float("nan")
    dirty = dirty.reshape(-1)
    plan = P.Plan(NSIDE, batch=BATCH, mode=mode, strategy=strategy)
    assert plan.strategy == strategy
    a0 = plan.analyze(clean)
    c0 = plan.power_spectrum(a0)
    a1 = plan.analyze(dirty)
    c1 = plan.power_spectrum(a1)
    torch.cuda.synchronize()
    a0, a1 = a0.cpu().numpy().reshape(BATCH, -1), a1.cpu().numpy().reshape(BATCH, -1)
    c0, c1 = c0.cpu().numpy().reshape(BATCH, -1), c1.cpu().numpy().reshape(BATCH, -1)
    plan.close()
    for v in range(BATCH):
        if v == BAD:
            assert np.isnan(a1[v]).any() and np.isnan(c1[v]).any()
        else:
            assert np.array_equal(a0[v], a1[v]), v
            assert np.array_equal(c0[v], c1[v]), v
    assert np.isfinite(a0).all()
