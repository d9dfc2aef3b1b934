#!/usr/bin/env python
"""Throughput of one MSM energy + force evaluation on one MI355X.

One step = one full evaluation (binning, short-range pairs, anterpolation,
restriction, lattice cutoff, top level, prolongation, interpolation,
reductions) of a 24,000-atom rigid 3-site water box (62.1 A cube, a = 12 A,
h = 2 A, cubic basis, 4 levels) whose float32 inputs are already resident in
HBM.  The metric is atom-evaluations per second (N / time per evaluation).
The plan is autotuned on the inputs first (untimed); the evaluation is timed
both replayed as a HIP graph and launched eagerly, and the faster is reported.

Prints one JSON line.  Besides the timed steps it reports
  * roofline: the dominant kernel's algorithmic FLOP rate against the FP32
    vector peak, timed with HIP events on the library's stream,
  * cpu_baseline: the FP64 CPU oracle on the same inputs on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3        # MI355X vector FP32 (256 CUs x 2.4 GHz x 256 FLOP/clk)
WORKLOADS = ("water24k", "water100k", "water1m", "cloud1k")


def make_system(name):
    from paper_1402_7216_amd import inputs
    return {"water24k": inputs.water_24k, "water100k": inputs.water_100k,
            "water1m": inputs.water_1m, "cloud1k": inputs.cloud_1k}[name]()


def traffic_for(kernel_key):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(kernel_key)
    if not rec:
        return None
    src = os.path.join(ROOT, "paper_1402_7216_amd", "csrc", "msm_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if rec.get("source_sha") != sha:
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(system, repeats):
    import oracle
    cores = len(os.sched_getaffinity(0))
    times = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        oracle.system_msm(system, threads=cores)
        times.append(time.perf_counter() - t0)
    t = statistics.median(times)
    return {"value": system.n / t, "unit": "atom-evals/s", "cores": cores, "kind": "oracle",
            "sample": f"full {system.n}-atom evaluation (energy, forces, potentials) in FP64, "
                      f"median of {repeats} runs, {t:.3f} s each"}


def batched_leg(msm, steps, warmup, autotune):
    """64 uneven water replicas (2,000-60,000 atoms, a = 10 A, h = 2 A): one
    batched graph replay against 64 single-system evaluations in sequence."""
    import torch
    from paper_1402_7216_amd import inputs
    reps = inputs.water_replicas(64)
    b = msm.batch_for(reps)
    x, y, z, q = msm.batch_to_device(reps)
    out = b.compute(x, y, z, q)
    torch.cuda.synchronize()
    b.check()
    best = b.autotune(x, y, z, q, trials=5)["best"] if autotune else None
    graph = b.graph(x, y, z, q, out)
    plans = [msm.plan_for(s) for s in reps]
    ins = [msm.to_device(s) for s in reps]
    outs = [p.compute(*i) for p, i in zip(plans, ins)]
    graphs = [msm.Graph(p, *i, o) for p, i, o in zip(plans, ins, outs)]

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    t_batch = timed(graph.launch)
    t_seq_graph = timed(lambda: [g.launch() for g in graphs])
    t_seq_eager = timed(lambda: [p.compute(*i, out=o) for p, i, o in zip(plans, ins, outs)])
    b.check()
    n = b.n
    return {"workload": "64 rigid-water replicas, 2k-60k atoms each (a = 10 A, h = 2 A, cubic)",
            "atoms": n, "ms_batched_graph": round(t_batch * 1e3, 4),
            "ms_64_sequential_graphs": round(t_seq_graph * 1e3, 4),
            "ms_64_sequential_eager": round(t_seq_eager * 1e3, 4),
            "atom_evals_per_s": n / t_batch,
            "speedup_vs_sequential_eager": round(t_seq_eager / t_batch, 3),
            "speedup_vs_sequential_graphs": round(t_seq_graph / t_batch, 3),
            "tuning": best}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="water24k", choices=WORKLOADS)
    ap.add_argument("--launch", default="best", choices=("best", "hipGraph", "eager"),
                    help="launch mode to time (best: time both, report the faster)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the plan's default tuning")
    ap.add_argument("--tuning", default=None,
                    help="JSON tuning to apply instead of autotuning, e.g. the config.tuning of an "
                         "earlier run (for profiler passes over the timed configuration)")
    ap.add_argument("--cpu-repeats", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-replica batched leg")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build evaluates each system on a single "
              "MI355X; run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1402_7216_amd import msm, workmodel

    torch.cuda.set_device(0)
    s = make_system(args.workload)
    plan = msm.plan_for(s)
    x, y, z, q = msm.to_device(s)
    out = plan.compute(x, y, z, q)
    torch.cuda.synchronize()
    plan.check()
    levels, glo, gn = plan.info()
    nodes = [int(np.prod(v)) for v in gn]
    if args.tuning:
        plan.tune(**json.loads(args.tuning))
    elif not args.no_autotune:
        plan.autotune(x, y, z, q, trials=40)

    graph = msm.Graph(plan, x, y, z, q, out)

    def timed(step, steps, warmup):
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / max(steps, 1)

    # both launch modes time the same evaluation; the faster one is reported
    modes = {"hipGraph replay": graph.launch, "eager": lambda: plan.compute(x, y, z, q, out=out)}
    if args.launch != "best":
        modes = {k: v for k, v in modes.items() if k.startswith(args.launch)}
    mode_sec = {k: timed(fn, args.steps, args.warmup) for k, fn in modes.items()}
    launch = min(mode_sec, key=mode_sec.get)
    sec = mode_sec[launch]
    plan.check()

    # per-stage kernel durations, HIP events on the library's stream (eager launches)
    plan.profile(True)
    stage_sum = {}
    n_prof = max(10, min(args.steps, 200))
    for _ in range(n_prof):
        plan.compute(x, y, z, q, out=out)
        for k, v in plan.stage_ms().items():
            stage_sum[k] = stage_sum.get(k, 0.0) + v
    plan.profile(False)
    stage_ms = {k: v / n_prof for k, v in stage_sum.items()}

    m = s.split_m or s.order // 2
    n_pairs = workmodel.count_pairs_within(s.pos64(), s.cutoff)
    work = workmodel.evaluation_work(s.n, n_pairs, nodes, s.cutoff, s.spacing, s.order, m)
    kernel_flops = {"short_range": work["short"], "lattice_cutoff": work["lattice"]}
    dom = max(kernel_flops, key=lambda k: stage_ms.get(k, 0.0))
    dom_s = stage_ms[dom] * 1e-3
    achieved = kernel_flops[dom] / dom_s / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "traffic": traffic_for(dom), "kernel": dom,
                "kernel_ms": round(stage_ms[dom], 5), "kernel_flop": kernel_flops[dom]}

    rec = {
        "metric": "MSM atom-evals/s (E+F)",
        "value": s.n / sec,
        "unit": "atom-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{s.name}: rigid 3-site water, 0.1 atoms/A^3" if s.name.startswith("water")
                   else s.name, "n_atoms": s.n, "cutoff": s.cutoff, "spacing": s.spacing,
                   "order": s.order, "levels": levels, "grid_sides": [int(v[0]) for v in gn],
                   "launch": launch, "tuning": plan.tuning()},
        "ms_per_launch_mode": {k: round(v * 1e3, 5) for k, v in mode_sec.items()},
        "roofline": roofline,
        "stages_ms": {k: round(v, 5) for k, v in stage_ms.items()},
        "algorithmic_tflops_per_step": round(work["total"] / sec / 1e12, 3),
        "algorithmic_flop_per_eval": work["total"],
        "unique_pairs": n_pairs,
    }
    if not args.no_batch:
        rec["batched"] = batched_leg(msm, max(5, min(args.steps // 10, 50)), 5, not args.no_autotune)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(s, args.cpu_repeats)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
