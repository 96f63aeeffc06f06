"""The autotuner's choices kept across processes (HP2SPH_TUNE_CACHE).

A first process autotunes a plan and appends its choices to the cache file
(one "key = fold pack ring threads schedules..." line, the key naming the
device, the mode and each group's nside, map count and strategy); a second
process creates a plan of the same shape without tuning and must start with
those choices; a third, after the line was rewritten with other valid
values, must start with the rewritten ones; a plan of another shape must
start with the defaults.  Each step runs in its own process, since a
process reads the file once, at its first plan creation."""

import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
sys.path.insert(0, sys.argv[1])
sys.path.insert(0, sys.argv[1] + "/tests")
import numpy as np
import torch
import paper_1904_10514_amd as P
from gpu_util import white_map
nsides = json.loads(sys.argv[2])
tune = sys.argv[3] == "tune"
plan = P.Plan(nsides, mode="f32_refine", strategy="tables")
if tune:
    maps = torch.from_numpy(np.concatenate([white_map(n, 2100 + i) for i, n in enumerate(nsides)])).cuda()
    plan.autotune(maps, reps=1)
    torch.cuda.synchronize()
print(json.dumps({"schedules": plan.schedules, "options": {o: plan.option(o) for o in P.OPTIONS}}))
plan.close()
"""


def _run(cache, nsides, tune):
    env = dict(os.environ, HP2SPH_TUNE_CACHE=cache)
    out = subprocess.run([sys.executable, "-c", CHILD, ROOT, json.dumps(nsides), "tune" if tune else "plain"],
                         env=env, cwd=ROOT, capture_output=True, text=True, timeout=240)
    assert out.returncode == 0, out.stderr[-2000:]
    return json.loads(out.stdout.strip().splitlines()[-1])


def test_tuning_cache_across_processes(tmp_path):
    cache = str(tmp_path / "tune.txt")
    shape = [16] * 9
    tuned = _run(cache, shape, True)
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith("v2/") and " = " in lines[0]
    key, vals = lines[0].split(" = ")
    assert key.endswith("/16x9t")
    v = [int(x) for x in vals.split()]
    o = tuned["options"]
    assert v[:4] == [o["fold_grid"], o["pack_maps"], o["ring_order"], o["ring_threads"]]
    assert [P_SCHEDULES.index(s) for s in tuned["schedules"]] == v[4:]
    # a new process starts with the tuned choices
    assert _run(cache, shape, False) == tuned
    # rewritten values (all valid, none the defaults) are taken as written
    want = {"fold_grid": 512, "pack_maps": 64, "ring_order": 2, "ring_threads": 512}
    sched = [3] * len(v[4:])
    with open(cache, "a") as fh:
        fh.write(key + " = " + " ".join(str(x) for x in [512, 64, 2, 512] + sched) + "\n")
    got = _run(cache, shape, False)
    assert got["options"] == want
    assert got["schedules"] == [P_SCHEDULES[3]] * len(sched)
    # another shape starts with the defaults
    other = _run(cache, [16] * 10, False)
    assert other["options"] == {"fold_grid": 0, "pack_maps": 32, "ring_order": 0, "ring_threads": 256}


P_SCHEDULES = ["xcd_round_robin", "xcd_balanced", "linear", "linear_rows"]
