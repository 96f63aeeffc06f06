"""GPU checks at the largest supported nside (2048, lmax 4096): the ring
transforms run 512-thread workgroups with 8192-point FFTs and the plan takes
the staged strategy (per-order tables would not fit).  The checks are the
exact-recovery property on order-1 fields (tests/gpu_util.py), which covers
the ring transform, pole, fit and packing of every l <= p, the synthesis and
the refinement; FP64 on a white-noise map against the oracle's values on
sampled orders up to m = 4096 (tests/golden/oplain_nside2048.txt, computed
offline: the oracle's dense colatitude fit takes minutes at this size),
which puts the Givens sweeps of every depth through a check; and, in
tests/test_gpu_equivariance.py, the exact equivariances at this size for
every order in both precision modes.  The last test runs the benchmark's own
shape at this nside (16 maps).
"""

import hashlib
import os

import numpy as np
import pytest
import torch

import paper_1904_10514_amd as P
from gpu_util import order_one_fields, rel_err

pytestmark = pytest.mark.gpu

NSIDE, BATCH = 2048, 2
LMAX = 2 * NSIDE


@pytest.fixture(scope="module")
def fields():
    maps, expect = order_one_fields(NSIDE, BATCH, 11)
    return torch.from_numpy(maps.reshape(-1)).cuda(), expect


def _golden2048():
    out = {"alm": {}}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "oplain_nside2048.txt")):
        w = line.split()
        if not w or w[0].startswith("#"):
            continue
        if w[0] == "sha256":
            out["sha256"] = w[1]
        elif w[0] == "alm":
            out["alm"][(int(w[1]), int(w[2]))] = complex(float(w[3]), float(w[4]))
    return out


def test_nside2048_f64_recovers_order_one_fields_and_matches_oracle(fields):
    """FP64, staged, on the two order-1 fields and on the white-noise map of
    tests/golden/oplain_nside2048.txt (the oracle's order-by-order route,
    written by make_oplain_nside2048.py), whose sampled orders m = 0 .. 4096
    (sweeps up to 2048 deep) must match to kappa p eps = 50 * 4096 * 1.1e-16."""
    dev, expect = fields
    import oracle as O
    import workloads as W
    g = _golden2048()
    white = W.random_map(O.npix(NSIDE), W.rng_for(14, 0))
    assert hashlib.sha256(np.ascontiguousarray(white).astype("<f8").tobytes()).hexdigest() == g["sha256"]
    batch = torch.cat([dev, torch.from_numpy(white).cuda()])
    del white
    plan = P.Plan(NSIDE, LMAX, batch=BATCH + 1, mode="f64")
    assert plan.strategy == "staged"
    a = plan.analyze(batch)
    torch.cuda.synchronize()
    a = a.cpu().numpy().reshape(BATCH + 1, -1)
    plan.close()
    e = rel_err(a[:BATCH], expect)
    keys = sorted(g["alm"])
    ref = np.array([g["alm"][k] for k in keys])
    got = np.array([a[BATCH][O.alm_index(l, m, LMAX)] for m, l in keys])
    eo = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    print(f"nside 2048, FP64: order-1 fields {e:.3e}; white noise vs oracle on sampled orders {eo:.3e}")
    assert e < 1e-12
    assert eo < 50 * 4096 * 1.1e-16


def test_nside2048_refinement_recovers_order_one_fields(fields):
    dev, expect = fields
    plan = P.Plan(NSIDE, LMAX, batch=BATCH, mode="f32_refine")
    assert plan.strategy == "staged"
    a1 = plan.analyze(dev)
    torch.cuda.synchronize()
    e1 = rel_err(a1.cpu().numpy().reshape(BATCH, -1), expect)
    # the refinement's synthesis is also the public synthesis: it must give
    # the fields back
    f = plan.synthesize(torch.from_numpy(expect.reshape(-1)).cuda())
    torch.cuda.synchronize()
    ef = rel_err(f.cpu().numpy(), dev.cpu().numpy())
    plan.close()
    print(f"order-1 fields, nside 2048 x 2: FP32 + refinement {e1:.3e}, synthesis {ef:.3e}")
    assert e1 < 1e-10
    assert ef < 1e-12


def test_nside2048_equal_weight_sampled_orders():
    """Equal-weight analysis (eq. healsph) at nside 2048 (staged: transposed
    evaluation + analysis sweeps, 8192-point longitude sums) on white noise,
    sampled orders of both maps against the oracle's per-order route; and the
    Jacobi residual |f - S a(k)| does not grow over two iterations."""
    import oracle as O
    import workloads as W
    npx = O.npix(NSIDE)
    maps = np.stack([W.random_map(npx, W.rng_for(12, v)) for v in range(BATCH)])
    dev = torch.from_numpy(maps.reshape(-1)).cuda()
    plan = P.Plan(NSIDE, LMAX, batch=BATCH, mode="equal_weight")
    assert plan.strategy == "staged"
    a = plan.analyze_iterative(dev, 0)
    torch.cuda.synchronize()
    a_h = a.cpu().numpy().reshape(BATCH, -1)
    orders = (0, 1, 3, 2047, 2048, 4095, 4096)
    worst = 0.0
    for v in range(BATCH):
        ref = O.equal_weight_columns(maps[v], NSIDE, orders, LMAX)
        scale = max(np.max(np.abs(r)) for r in ref.values())
        for m, r in ref.items():
            idx = np.array([O.alm_index(l, m, LMAX) for l in range(m, LMAX + 1)])
            worst = max(worst, np.max(np.abs(a_h[v, idx] - r)) / scale)
    print(f"equal weight nside 2048 x 2, sampled: {worst:.3e}")
    # staged: up to p/2 sweeps on each coefficient and 2 nside-term sums,
    # p eps sqrt(2 nside) = 4096 * 1.1e-16 * 64 = 2.9e-11
    assert worst < 2.9e-11
    norms = []
    for k in range(3):
        ak = plan.analyze_iterative(dev, k)
        norms.append(float(torch.linalg.vector_norm(dev - plan.synthesize(ak))))
        del ak
    print("residual norms:", norms)
    assert norms[1] <= norms[0] * (1 + 1e-12) and norms[2] <= norms[1] * (1 + 1e-12)
    plan.close()


def test_nside2048_batch16_bench_shape():
    """The nside-2048 benchmark configuration itself: 16 maps, lmax 4096, the
    FP32 + refinement plan (its FP64 ring transform and synthesis included)
    with the default schedules (`linear_rows` for the staged GEMMs, what the
    bench's autotuner picks at this shape; the tuner itself is tested in
    test_gpu_schedule.py); on order-1 fields (recovered exactly for every
    l <= p) it must return the input coefficients of all 16 maps.  (FP64 at
    this nside is checked on 2 maps above: each nside-2048 plan takes about a
    minute to set up.)"""
    batch = 16
    maps, expect = order_one_fields(NSIDE, batch, 14)
    dev = torch.from_numpy(maps.reshape(-1)).cuda()
    del maps
    for mode, tol in (("f32_refine", 1e-10),):
        plan = P.Plan(NSIDE, LMAX, batch=batch, mode=mode)
        assert plan.strategy == "staged"
        assert plan.schedules == ["linear_rows"] * len(plan.schedules)
        a = plan.analyze(dev)
        torch.cuda.synchronize()
        e = rel_err(a.cpu().numpy().reshape(batch, -1), expect)
        print(f"order-1 fields, nside 2048 x 16, {mode} (schedules {plan.schedules}): {e:.3e}")
        plan.close()
        del a
        assert e < tol
