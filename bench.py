#!/usr/bin/env python3
"""Benchmark of HP2SPH analysis on one MI355X.

Workload: a batch of 64 HEALPix maps, nside 1024 (12,582,912 pixels each),
lmax 2048, seeded CMB-like inputs: Gaussian a_lm with
C_l = exp(-l(l+1) s^2) / (l(l+1)), s = 0.005, synthesised on the GPU, plus
white pixel noise of standard deviation 1e-3 of each map's rms (seeded).
Inputs are resident in HBM before the timed region.

One step = one pass of the whole analysis path over the batch: the per-ring
transforms, pole values, colatitude fit, Givens sweeps and packing of a_lm
(for the FP32+refinement mode: FP64 ring transforms, FP32 colatitude fit and
Legendre conversion, FP64 synthesis coefficients, the residual in ring-Fourier
space, FP32 analysis of the residual, FP64 accumulation), then C_l.  The headline
value is maps/s of batched FP32+refinement; plain FP64 is timed beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
Prints one JSON line.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "maps analysed/s at nside={nside}, L={lmax}: batched FP32+refine vs plain FP64"

# MI355X published peaks.  The VALU figure for FP32 (157.3) counts packed
# FP32 instructions, which the library is compiled never to emit (packed-fp32-ops off):
# non-packed FP32 issues at the FP64 VALU rate, 78.6 TFLOP/s.
PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"mfma": {"f32": 157.3, "f64": 78.6}, "alu": {"f32": 78.6, "f64": 78.6}}


def block_dims(nside):
    p = 2 * nside
    lmin = [0, 1, 1, 2]
    nl = [(p - lm) // 2 + 1 for lm in lmin]
    nk = [p // 2 + 1, p // 2 + 1, p // 2, p // 2]
    return p, nl, nk


def sweep_rotations(nside, nmaps):
    """Real Givens rotations per sweep launch (each 6 flops)."""
    _, nl, nk = block_dims(nside)
    tot = 0
    for b in range(4):
        for kk in range(nk[b]):
            # sweeps t = 1..kk, each over positions l' = t .. nl-1
            tot += kk * nl[b] - kk * (kk + 1) // 2
    return 2 * nmaps * tot


def order_gemm_flops(nside, nmaps, synthesis):
    """Flops of the per-order GEMMs: for block b and mode k' a (nl-k') x K' matrix
    times 2*nmaps columns; K' skips the polar rings that cannot carry the mode
    (analysis) or is the 2*nside rings (synthesis)."""
    p, nl, nk = block_dims(nside)
    K = 2 * nside + 1
    tot = 0
    for b in range(4):
        kpar = b >> 1
        for kk in range(nk[b]):
            m = 2 * kk + kpar
            h0 = 0 if m == 0 else (m + 1) // 2
            kd = 2 * nside if synthesis else K - h0
            tot += 2 * (nl[b] - kk) * kd * 2 * nmaps
    return tot


def stage_work(stage, nside, nmaps, tsize, strategy="staged", mode="f64"):
    """(kind, amount) algorithmic work of one launch: ('flop', n) or ('byte', n)."""
    p, nl, nk = block_dims(nside)
    K = 2 * nside + 1
    N = [nmaps * 2 * nk[0], nmaps * 2 * nk[2]]
    npix = 12 * nside * nside * nmaps
    if stage in ("gemm_analysis", "gemm_synthesis", "gemm_adjoint") and strategy == "tables":
        return "flop", order_gemm_flops(nside, nmaps, stage != "gemm_analysis")
    if stage == "gemm_analysis":
        return "flop", sum(2 * nl[b] * K * N[b >> 1] for b in range(4))
    if stage == "gemm_synthesis":
        return "flop", sum(2 * nl[b] * K * N[b >> 1] for b in range(4))
    if stage == "gemm_adjoint":
        return "flop", sum(2 * nl[b] * (K - 1) * N[b >> 1] for b in range(4))
    if stage in ("sweep_analysis", "sweep_synthesis"):
        return "flop", 6 * sweep_rotations(nside, nmaps)
    rows = 2 * nside * (N[0] + N[1]) * 2   # values of Dsym rows 1..2 nside, both D+ and D-
    if stage == "ring_forward":
        return "byte", npix * 8 + rows * tsize
    if stage == "ring_adjoint":
        return "byte", npix * 8 + rows * 8
    if stage == "ring_inverse":
        return "byte", rows * 8 + npix * 8
    if stage == "residual_fold":
        # refinement: read Df and the synthesis output (FP64), write FP32;
        # equal-weight iteration: read Wf and the synthesis output, write Wr (FP64)
        return "byte", rows * (8 + 8 + (8 if mode == "equal_weight" else 4))
    u_vals = sum(nl[b] * N[b >> 1] for b in range(4))   # values of the U blocks (rectangle)
    n_alm = (p + 1) * (p + 2) // 2 * nmaps                # a_l^m, m <= l <= p: the live U entries
    alm_bytes = n_alm * 16
    if stage == "pack":
        # the refinement packs a0 + correction (two U reads); so does every
        # Jacobi update of the staged equal-weight analysis but the first pack
        n_in = 2 if mode == "f32_refine" or (mode == "equal_weight" and strategy != "tables") else 1
        return "byte", n_in * n_alm * 2 * tsize + alm_bytes
    if stage == "pole":
        # reads the three ring rows' (k = 0, real) entries of every map, writes row 0 of the four blocks
        return "byte", 3 * 2 * nmaps * tsize + sum(N[b >> 1] for b in range(4)) * tsize
    if stage == "unpack":
        if mode == "f32_refine":
            # FP32 a0 widened to FP64: reads the live FP32 pairs; writes the live
            # triangle (per-order tables, rows l >= m only) or the whole U
            # rectangle (staged sweeps)
            return "byte", n_alm * 2 * 4 + (n_alm * 16 if strategy == "tables" else u_vals * 8)
        if mode == "equal_weight" and strategy == "tables":   # a += A r in the U layout
            return "byte", 3 * n_alm * 16
        return "byte", alm_bytes + u_vals * 8
    if stage == "cl":
        return "byte", (p + 1) * (p + 2) // 2 * 16 * nmaps
    return "byte", 0


def stage_bound(stage):
    if stage.startswith("gemm"):
        return "mfma"
    if stage.startswith("sweep"):
        return "alu"
    return "hbm"


def stage_dtype(stage, mode):
    if mode == "equal_weight":
        return "f64"
    if stage == "ring_forward":   # FP64 in every mode
        return "f64"
    if mode == "f64" or stage in ("sweep_synthesis", "gemm_synthesis", "ring_inverse", "unpack", "cl",
                                  "residual_fold"):
        return "f64"
    return "f32"


def roofline(stage, mode, nside, nmaps, ms_total, launches, strategy="staged"):
    dt = stage_dtype(stage, mode)
    kind, amount = stage_work(stage, nside, nmaps, 4 if dt == "f32" else 8, strategy, mode)
    avg_s = ms_total / launches / 1e3
    bound = stage_bound(stage)
    if bound == "hbm":
        achieved = amount / avg_s / 1e9
        peak, unit = PEAK_HBM_GBS, "GB/s"
    else:
        achieved = amount / avg_s / 1e12
        peak, unit = PEAK_TFLOPS[bound][dt], "TFLOP/s"
    return {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
            "traffic": measured_traffic(stage, dt, nside, nmaps, strategy), "kernel": stage, "dtype": dt,
            "strategy": strategy,
            "avg_launch_ms": avg_s * 1e3,
            "work_per_launch": amount, "work_unit": kind}


def uneven_roofline(stage, mode, counts, ms_total, launches, strategy):
    """roofline() of a stage launched once over several nside groups
    (counts: nside -> maps): the algorithmic work of a launch is the sum over
    the groups.  No counter summary covers these launches (traffic null)."""
    dt = stage_dtype(stage, mode)
    kind, amount = "byte", 0
    for ns, nm in counts.items():
        kind, a = stage_work(stage, ns, nm, 4 if dt == "f32" else 8, strategy, mode)
        amount += a
    avg_s = ms_total / launches / 1e3
    bound = stage_bound(stage)
    if bound == "hbm":
        achieved, peak, unit = amount / avg_s / 1e9, PEAK_HBM_GBS, "GB/s"
    else:
        achieved, peak, unit = amount / avg_s / 1e12, PEAK_TFLOPS[bound][dt], "TFLOP/s"
    return {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
            "traffic": None, "kernel": stage, "dtype": dt, "strategy": strategy, "avg_launch_ms": avg_s * 1e3,
            "launches": launches, "work_per_launch": amount, "work_unit": kind}


def measured_traffic(stage, dtype, nside, nmaps, strategy):
    """HBM bytes per launch from the committed counter runs (profiles/), scaled
    by the copy-kernel calibration; None if the kernels changed since then or
    the workload differs."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_nside{nside}_L{2 * nside}_b{nmaps}.json")
    try:
        with open(path) as fh:
            js = json.load(fh)
        src = os.path.join(ROOT, "paper_1904_10514_amd", "csrc", "kernels.hip")
        with open(src, "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != js["kernels_hip_sha256"]:
                return None
        if js["workload"] != {"nside": nside, "lmax": 2 * nside, "batch": nmaps, "strategy": strategy}:
            return None
        e = js["stages"].get(f"{stage}/{dtype}")
        # read_bytes / write_bytes are already means over the stage's
        # dispatches in the counter runs (two for the FP32 analysis GEMMs)
        return None if e is None else e["read_bytes"] + e["write_bytes"]
    except (OSError, KeyError, ValueError):
        return None


def input_recipe(nside):
    """(workloads config id, relative noise, description) of the benchmark maps:
    the nside-2048 configuration (config 4: a bump five times the baseline at
    l = 220, width 60, beam s = 0.002, no noise); otherwise the nside-1024
    recipe (config 2: beam s = 0.005, plus white noise of 1e-3 of each map's rms)."""
    if nside == 2048:
        return 4, 0.0, ("seeded Gaussian a_lm, C_l=[1/(l(l+1))][1+4 exp(-(l-220)^2/(2*60^2))] exp(-l(l+1)s^2), "
                        "s=0.002, GPU FP64 synthesis, no noise")
    return 2, 1e-3, ("seeded Gaussian a_lm, C_l=exp(-l(l+1)s^2)/(l(l+1)), s=0.005, GPU FP64 synthesis, "
                     "+ white noise 1e-3 x map rms")


def make_inputs(torch, P, W, nside, nmaps):
    """Seeded CMB-like maps (GPU FP64 synthesis of seeded a_lm), plus white
    noise where the recipe has it (input_recipe)."""
    import numpy as np
    lmax = 2 * nside
    cfg, noise_rel, _ = input_recipe(nside)
    cl = W.spectrum(cfg, lmax)
    alm = np.concatenate([W.draw_alm(cl, lmax, W.rng_for(cfg, i)) for i in range(nmaps)])
    syn = P.Plan(nside, lmax, batch=nmaps, mode="f64", strategy="staged")
    maps = syn.synthesize(torch.from_numpy(alm).cuda())
    torch.cuda.synchronize()
    syn.close()
    del syn
    if noise_rel > 0:
        m2 = maps.view(nmaps, -1)
        rms = m2.pow(2).mean(dim=1).sqrt()
        g = torch.Generator(device="cuda")
        g.manual_seed(1904 * 1000003 + 10514 * 1009 + cfg)
        noise = torch.randn(m2.shape, generator=g, device="cuda", dtype=torch.float64)
        m2.add_(noise * (noise_rel * rms[:, None]))
        del noise
    torch.cuda.synchronize()
    return maps


P_OPTIONS = ("fold_grid", "pack_maps", "ring_order", "ring_threads")


def autotune(plan, maps, out, enabled):
    """Set-up step outside the timed region: the plan's autotuner picks the
    GEMM workgroup schedules and the launch options (fold grid, pack tile
    shape) on these maps."""
    def options():
        return {name: plan.option(name) for name in P_OPTIONS}
    if not enabled:
        return {"enabled": False, "schedules": plan.schedules, "options": options()}
    t0 = time.perf_counter()
    ms, _ = plan.autotune(maps, reps=3, out=out)
    return {"enabled": True, "schedules": plan.schedules, "options": options(), "best_ms": ms,
            "seconds": time.perf_counter() - t0}


def map0_sha256(maps, npix):
    """SHA-256 of the first input map (FP64, little-endian bytes), recorded
    with the bench line so a run's inputs can be compared across runs."""
    import hashlib
    return hashlib.sha256(maps[:npix].cpu().numpy().astype("<f8").tobytes()).hexdigest()


def time_mode(torch, P, maps, nside, nmaps, mode, steps, warmup, strategy, tune=True):
    t0 = time.perf_counter()
    plan = P.Plan(nside, 2 * nside, batch=nmaps, mode=mode, strategy=strategy)
    setup_s = time.perf_counter() - t0
    alm = torch.empty(plan.alm_total, dtype=torch.complex128, device="cuda")
    cl = torch.empty(plan.cl_total, dtype=torch.float64, device="cuda")
    tuned = autotune(plan, maps, alm, tune)
    for _ in range(warmup):
        plan.analyze(maps, out=alm)
        plan.power_spectrum(alm, out=cl)
    torch.cuda.synchronize()
    plan.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.analyze(maps, out=alm)
        plan.power_spectrum(alm, out=cl)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    plan.profile(False)
    prof = plan.profile_read()
    return plan, alm, cl, dt, setup_s, prof, tuned


def host_info():
    """Host facts recorded with the CPU baseline: logical CPUs, the CPU model
    (/proc/cpuinfo), and the BLAS library numpy and scipy use with its threads."""
    info = {"nproc": os.cpu_count()}
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        info["blas"] = [{k: i.get(k) for k in ("internal_api", "version", "num_threads", "threading_layer")}
                        for i in threadpool_info() if i.get("user_api") == "blas"]
    except Exception:
        info["blas"] = None
    return info


def cpu_baseline(f_host, nside, nsample=48, full=False):
    """The oracle on a bounded sample: one map through the Fourier-space route
    of Algorithm 1 for `nsample` evenly spaced orders m, scaled to a map.  With
    `full`, also one whole map through O_plain (the spatial route, Algorithm 1
    literally) and through O_ref (two analyses and one exact synthesis), each
    timed once (minutes at nside 1024)."""
    import numpy as np
    import oracle as O
    from oracle import hp2sph as OH
    hinfo = host_info()
    cores = max([b.get("num_threads") or 1 for b in (hinfo.get("blas") or [])] + [1])
    lmax = 2 * nside
    t0 = time.perf_counter()
    OH._lsq(nside)                      # colatitude QR: set-up, independent of the map
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    OH.ring_coefficients(f_host, nside)
    OH.pole_values(f_host, nside)
    t_rings = time.perf_counter() - t0
    ms = sorted(set(np.linspace(0, lmax, nsample).astype(int).tolist()))
    t0 = time.perf_counter()
    O.analyze_columns(f_host, nside, ms, lmax)
    t_cols = time.perf_counter() - t0
    per_col = max(t_cols - t_rings, 0.0) / len(ms)
    per_map = t_rings + per_col * (lmax + 1)
    out = {"value": 1.0 / per_map, "unit": "maps/s", "cores": int(cores), "kind": "oracle",
           "sample": (f"one nside-{nside} map of the workload through the FP64 oracle's Fourier-space "
                      f"route (ring DFTs, pole fit, dense-QR colatitude fit, Gauss-Legendre projection) "
                      f"for {len(ms)} evenly spaced orders of {lmax + 1}, scaled to all orders; the "
                      f"colatitude QR set-up ({t_setup:.1f} s) excluded; the refined oracle O_ref costs two such "
                      f"analyses plus one exact synthesis"),
           "seconds_timed": t_cols + t_rings, "host": hinfo}
    if full:
        t0 = time.perf_counter()
        a0 = O.analyze(f_host, nside, lmax)
        t_plain = time.perf_counter() - t0
        t0 = time.perf_counter()
        s0 = O.synthesize(a0, nside, lmax)
        t_syn = time.perf_counter() - t0
        t0 = time.perf_counter()
        O.analyze(f_host - s0, nside, lmax)
        t_second = time.perf_counter() - t0
        out["full_map_s"] = {"o_plain": t_plain, "o_synth": t_syn, "o_ref": t_plain + t_syn + t_second}
    return out


def uneven_main(args):
    """The batching form: 256 maps of seeded uneven nside in {64, 128, 256, 512},
    lmax = 2 nside, C_l = l^-2 exp(-l(l+1) s^2), one plan for the whole batch.
    Prints its own JSON line (a secondary measurement, not the headline)."""
    import numpy as np
    import torch
    import workloads as W
    import paper_1904_10514_amd as P
    nsides = [int(v) for v in W.uneven_nsides(256, 3)]
    lmaxs = [2 * v for v in nsides]
    counts = {int(n): nsides.count(n) for n in sorted(set(nsides))}
    alm = np.concatenate([W.draw_alm(W.spectrum(3, L), L, W.rng_for(3, i)) for i, L in enumerate(lmaxs)])
    syn = P.Plan(nsides, lmaxs, mode="f64", strategy="staged")
    maps = syn.synthesize(torch.from_numpy(alm).cuda())
    torch.cuda.synchronize()
    syn.close()
    del syn
    res = {}
    for mode in [m for m in args.modes.split(",") if m]:
        t0 = time.perf_counter()
        plan = P.Plan(nsides, lmaxs, mode=mode, strategy=args.strategy)
        setup = time.perf_counter() - t0
        out = torch.empty(plan.alm_total, dtype=torch.complex128, device="cuda")
        cl = torch.empty(plan.cl_total, dtype=torch.float64, device="cuda")
        tuned = autotune(plan, maps, out, not args.no_autotune)
        for _ in range(args.warmup):
            plan.analyze(maps, out=out)
            plan.power_spectrum(out, out=cl)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.analyze(maps, out=out)
            plan.power_spectrum(out, out=cl)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        # the same step as one graph launch (the analyze and C_l calls only
        # enqueue kernels, so they capture into a HIP graph)
        ref = out.clone()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            plan.analyze(maps, out=out)
            plan.power_spectrum(out, out=cl)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            plan.analyze(maps, out=out)
            plan.power_spectrum(out, out=cl)
        graph.replay()
        torch.cuda.synchronize()
        if not torch.equal(out, ref):
            raise RuntimeError("graph replay differs from the eager analysis")
        t0 = time.perf_counter()
        for _ in range(args.steps):
            graph.replay()
        torch.cuda.synchronize()
        dtg = time.perf_counter() - t0
        del graph
        # per-stage times (HIP events) of as many steps again; each stage is one
        # launch over the four nside groups, so its work is the groups' sum
        plan.profile(True)
        for _ in range(args.steps):
            plan.analyze(maps, out=out)
        torch.cuda.synchronize()
        plan.profile(False)
        prof = plan.profile_read()
        stages = {st: uneven_roofline(st, mode, counts, ms, n, plan.strategy)
                  for st, (ms, n) in prof.items() if n}
        dom = max((st for st in stages if st.startswith("gemm")), key=lambda st: stages[st]["avg_launch_ms"])
        res[mode] = {"maps_per_s": len(nsides) * args.steps / dt, "ms_per_step": 1e3 * dt / args.steps,
                     "graph_maps_per_s": len(nsides) * args.steps / dtg, "graph_ms_per_step": 1e3 * dtg / args.steps,
                     "setup_s": setup, "strategy": plan.strategy, "autotune": tuned, "roofline": stages[dom],
                     "stages": {st: {"ms_per_step": v["avg_launch_ms"] * v["launches"] / args.steps,
                                     "launches": v["launches"], "achieved": v["achieved"], "unit": v["unit"],
                                     "frac": v["frac"]} for st, v in stages.items()}}
        print(f"[bench] uneven {mode}: {1e3 * dt / args.steps:.2f} ms/step, as one graph launch "
              f"{1e3 * dtg / args.steps:.2f} ms/step", file=sys.stderr, flush=True)
        plan.close()
        del plan
    head = res.get("f32_refine") or next(iter(res.values()))
    print(json.dumps({"metric": "maps analysed/s, uneven batch (batching form)", "value": head["maps_per_s"],
                      "unit": "maps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
                      "vs_baseline": None, "dtype": "f32+f64" if "f32_refine" in res else "f64", "data": "synthetic",
                      "roofline": head["roofline"],
                      "config": {"workload": "uneven_b256_nside64-512", "batch": len(nsides), "nside_counts": counts,
                                 "lmax": "2 nside",
                                 "input": "seeded Gaussian a_lm, C_l=l^-2 exp(-l(l+1)s^2), s=0.005, GPU FP64 synthesis",
                                 "input_sha256_map0": map0_sha256(maps, 12 * nsides[0] * nsides[0])},
                      "modes": res}), flush=True)


def equal_weight_main(args):
    """The equal-weight analysis with Jacobi iterations (eqs. healsph, uzawa;
    the method the paper compares HP2SPH with) on the headline inputs: 64 maps
    of nside 1024, lmax 2048, niter = 3.  Prints its own JSON line (a secondary
    measurement, not the headline)."""
    import torch
    import workloads as W
    import paper_1904_10514_amd as P
    nside, nmaps, niter = args.nside, args.batch, args.niter
    lmax = 2 * nside
    print(f"[bench] building inputs: {nmaps} maps, nside {nside}", file=sys.stderr, flush=True)
    maps = make_inputs(torch, P, W, nside, nmaps)
    t0 = time.perf_counter()
    plan = P.Plan(nside, lmax, batch=nmaps, mode="equal_weight", strategy=args.strategy)
    setup_s = time.perf_counter() - t0
    alm = torch.empty(plan.alm_total, dtype=torch.complex128, device="cuda")
    # the autotuner times hp2sph_analyze, i.e. 3 Jacobi iterations
    tuned = autotune(plan, maps, alm, not args.no_autotune and niter == 3)
    for _ in range(args.warmup):
        plan.analyze_iterative(maps, niter, out=alm)
    torch.cuda.synchronize()
    plan.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.analyze_iterative(maps, niter, out=alm)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    plan.profile(False)
    prof = plan.profile_read()
    stages = {}
    for st, (ms, n) in prof.items():
        if n:
            rl = roofline(st, "equal_weight", nside, nmaps, ms, n, plan.strategy)
            stages[st] = {"ms_per_step": ms / args.steps, "launches": n, "achieved": rl["achieved"],
                          "unit": rl["unit"], "frac": rl["frac"]}
    dom = max((st for st in stages if st.startswith("gemm")), key=lambda st: stages[st]["ms_per_step"])
    rl = roofline(dom, "equal_weight", nside, nmaps, prof[dom][0], prof[dom][1], plan.strategy)
    rl["traffic"] = None
    print(f"[bench] equal weight, {niter} Jacobi iterations: {1e3 * dt / args.steps:.2f} ms/step, "
          f"set-up {setup_s:.1f} s", file=sys.stderr, flush=True)
    print(json.dumps({"metric": f"maps analysed/s at nside={nside}, L={lmax}: equal-weight analysis + "
                                f"{niter} Jacobi iterations (FP64)",
                      "value": nmaps * args.steps / dt, "unit": "maps/s", "n_gpus": 1, "steps": args.steps,
                      "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
                      "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
                      "config": {"workload": f"equal_weight_nside{nside}_L{lmax}_b{nmaps}", "nside": nside,
                                 "lmax": lmax, "batch": nmaps, "niter": niter, "strategy": plan.strategy,
                                 "input_sha256_map0": map0_sha256(maps, 12 * nside * nside)},
                      "setup_s": setup_s, "autotune": tuned, "roofline": rl, "stages": stages}), flush=True)
    plan.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--nside", type=int, default=1024)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-full", action="store_true",
                    help="also time one whole map through the oracle's O_plain and O_ref (minutes at nside 1024)")
    ap.add_argument("--strategy", default="auto", choices=["auto", "staged", "tables"])
    ap.add_argument("--modes", default="f32_refine,f64",
                    help="precision modes to time; the headline is f32_refine (profiling runs may pick one)")
    ap.add_argument("--workload", default="headline", choices=["headline", "uneven", "equal_weight"],
                    help="headline: 64 maps of nside 1024; uneven: 256 maps of nside 64..512; equal_weight: "
                         "the equal-weight analysis with Jacobi iterations on the headline inputs (secondary)")
    ap.add_argument("--niter", type=int, default=3, help="Jacobi iterations of the equal_weight workload")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default GEMM schedules instead of running the plan's autotuner at set-up")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (maps of a batch "
              "are independent and would be sharded across GPUs with no communication).", file=sys.stderr)
        sys.exit(2)
    if args.workload == "uneven":
        uneven_main(args)
        return
    if args.workload == "equal_weight":
        equal_weight_main(args)
        return

    import numpy as np
    import torch
    import workloads as W
    import paper_1904_10514_amd as P

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    nside, nmaps = args.nside, args.batch
    lmax = 2 * nside
    print(f"[bench] building inputs: {nmaps} maps, nside {nside}", file=sys.stderr, flush=True)
    maps = make_inputs(torch, P, W, nside, nmaps)

    modes = [m for m in args.modes.split(",") if m]
    results = {}
    for mode in modes:
        print(f"[bench] timing {mode}", file=sys.stderr, flush=True)
        plan, alm, cl, dt, setup_s, prof, tuned = time_mode(torch, P, maps, nside, nmaps, mode, args.steps,
                                                            args.warmup, args.strategy, not args.no_autotune)
        results[mode] = {"plan": plan, "alm": alm, "cl": cl, "dt": dt, "setup_s": setup_s, "prof": prof,
                         "strategy": plan.strategy, "autotune": tuned}
        print(f"[bench] {mode}: {1e3 * dt / args.steps:.2f} ms/step, set-up {setup_s:.1f} s, "
              f"schedules {tuned['schedules']}", file=sys.stderr, flush=True)

    head = results.get("f32_refine") or results[modes[0]]
    head_mode = "f32_refine" if "f32_refine" in results else modes[0]
    f64 = results.get("f64")
    ms_step = 1e3 * head["dt"] / args.steps
    value = nmaps * args.steps / head["dt"]
    f64_value = nmaps * args.steps / f64["dt"] if f64 else None

    # dominant kernel of the headline mode, against its binding roofline
    prof = head["prof"]
    dom = max(prof, key=lambda k: prof[k][0])
    roof = roofline(dom, head_mode, nside, nmaps, prof[dom][0], prof[dom][1], head["strategy"])
    stages = {}
    for mode in modes:
        pr = results[mode]["prof"]
        stages[mode] = {k: {"ms_per_step": v[0] / args.steps, "launches": v[1],
                            **{kk: vv for kk, vv in roofline(k, mode, nside, nmaps, v[0], v[1],
                                                             results[mode]["strategy"]).items()
                               if kk in ("achieved", "unit", "frac")}}
                        for k, v in pr.items() if v[1] > 0}

    # FP32+refine against the FP64 GPU result (the method change of the
    # refinement, R12) and against the same recipe in FP64 on the GPU,
    # a64 + A64(f - S64 a64) (the FP64 path and synthesis are parity-tested
    # against the oracle; tests/test_gpu_headline_accuracy.py checks the
    # FP32+refine result against the oracle's refined analysis itself)
    vs_plain = vs_recipe = None
    if f64 is not None and head is not f64:
        def errs(a, ref):
            c = f64["plan"].power_spectrum(a).view(nmaps, -1)
            cr = f64["plan"].power_spectrum(ref).view(nmaps, -1)
            rel = ((c - cr).abs()[:, 2:] / cr[:, 2:]).amax(dim=0)
            da = (a - ref).abs().view(nmaps, -1).amax(dim=1) / ref.abs().view(nmaps, -1).amax(dim=1)
            # degrees whose C_l stays above 1e-12 of the largest (every map):
            # beyond them a noiseless beamed spectrum falls below FP64
            # rounding of the sums and a relative error carries no meaning
            big = (cr[:, 2:] >= 1e-12 * cr[:, 2:].amax(dim=1, keepdim=True)).all(dim=0)
            l_cut = int(2 + (big.nonzero().max() if bool(big.any()) else 0))
            return {"max_abs_da_over_max_a": float(da.max()), "max_rel_dcl_l_ge_2": float(rel.max()),
                    "l_cut": l_cut, "max_rel_dcl_2_to_l_cut": float(rel[:l_cut - 1].max()),
                    "median_over_l_of_max_rel_dcl": float(rel.median()),
                    "rel_dcl_by_band": {f"{lo}-{hi}": float(rel[lo - 2:hi - 1].max())
                                        for lo, hi in ((2, 100), (100, 500), (500, 1000), (1000, 1500), (1500, lmax))}}
        a32, a64 = head["alm"], f64["alm"]
        vs_plain = errs(a32, a64)
        p64 = f64["plan"]
        ref = a64 + p64.analyze(maps - p64.synthesize(a64))
        vs_recipe = errs(a32, ref)
        del ref
        torch.cuda.synchronize()

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        f0 = maps[:12 * nside * nside].cpu().numpy()
        cpu = cpu_baseline(f0, nside, full=args.cpu_full)

    line = {
        "metric": METRIC.format(nside=nside, lmax=lmax),
        "value": value,
        "unit": "maps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"nside{nside}_L{lmax}_b{nmaps}", "nside": nside, "lmax": lmax, "batch": nmaps,
                   "mode": head_mode, "strategy": head["strategy"], "input_sha256_map0": map0_sha256(maps, 12 * nside * nside),
                   "input": input_recipe(nside)[2]},
        "f64_maps_per_s": f64_value,
        "f64_ms_per_step": 1e3 * f64["dt"] / args.steps if f64 else None,
        "setup_s": {m: results[m]["setup_s"] for m in results},
        "strategy": {m: results[m]["strategy"] for m in results},
        "autotune": {m: results[m]["autotune"] for m in results},
        "roofline": roof,
        "stages": stages,
        "f32refine_vs_gpu_f64": vs_plain,
        "f32refine_vs_gpu_f64_refined_recipe": vs_recipe,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
