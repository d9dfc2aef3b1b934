#!/usr/bin/env python
"""Throughput of one MSM energy + force evaluation on one MI355X.

One step = one full evaluation (binning, short-range pairs, anterpolation,
restriction, lattice cutoff, top level, prolongation, interpolation,
reductions) whose float32 inputs are already resident in HBM.  The headline
workload is the largest single-GPU system: 999,999 atoms of rigid 3-site
water (215.4 A cube, a = 12 A, h = 2.5 A, quintic basis, 5 levels).  The
metric is atom-evaluations per second (N / time per evaluation).  The plan is
autotuned on the inputs first (untimed); the evaluation is timed both replayed
as a HIP graph and launched eagerly, and the faster is reported.  Each timed
step is bracketed by HIP events, so the line carries the median step beside
the mean of the K-step window.

Prints one JSON line.  Besides the timed steps it reports
  * roofline: the dominant kernel's algorithmic FLOP rate against the FP32
    vector peak, its launches timed with HIP events on the stream they run on
    in the timed schedule (K more evaluations), and alone (stages in order);
  * parity: the timed configuration's forces, potentials and energy against
    the FP64 CPU oracle on the same inputs;
  * cpu_baseline: that oracle run, timed on the host cores (plus one-thread
    times of the 1,000-atom cloud and the 24,000-atom water box);
  * coarse_propagators / cheap_msm_propagators: the cheap pair methods
    (cutoff, shifted-force smoothed cutoff, Wolf) and MSM with a 4x coarser
    finest grid or a 6 A cutoff on the same inputs, as parareal coarse
    functions G: time, Q_F/G against the timed evaluation F, and their
    force / energy distance from F;
  * extras: a parareal window (batched MSM fine propagator, shifted-force
    coarse propagator) on a 27,000-ion cluster against sequential steps,
    the 24,000-atom box, the 100,000-atom box through the
    differentiable path (energy, then backward), and the 64-replica batch
    (forward, and forward + backward) against 64 sequential evaluations.
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

PEAK_FP32_TFLOPS = 157.3        # MI355X vector FP32 (256 CUs x 2.4 GHz x 256 FLOP/clk, packed)
WORKLOADS = ("water1m", "water24k", "water100k", "cloud1k")


def make_system(name):
    from paper_1402_7216_amd import inputs
    return {"water24k": inputs.water_24k, "water100k": inputs.water_100k,
            "water1m": inputs.water_1m, "cloud1k": inputs.cloud_1k}[name]()


def describe_workload(s):
    if s.name == "water1m":
        return "water1m: 999,999-atom rigid 3-site water box, 0.1 atoms/A^3"
    if s.name.startswith("water"):
        return f"{s.name}: {s.n}-atom rigid 3-site water box, 0.1 atoms/A^3"
    return s.name


def traffic_for(kernel_key, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(workload, {}).get(kernel_key)
    if not rec:
        return None
    src = os.path.join(ROOT, "paper_1402_7216_amd", "csrc", "msm_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if rec.get("source_sha") != sha:
        return None
    return rec.get("bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def event_timed(torch, step, steps, warmup):
    """W untimed steps, then K steps bracketed by synchronisation, each step
    between two HIP events on the current stream.  Returns (mean s, median s)."""
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(steps):
        step()
        ev[k + 1].record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / max(steps, 1)
    per = [ev[k].elapsed_time(ev[k + 1]) * 1e-3 for k in range(steps)]
    return max(wall, sum(per) / max(steps, 1)), statistics.median(per)


def parity(out, ref):
    import numpy as np
    f = out["f"].double().cpu().numpy()
    phi = out["phi"].double().cpu().numpy()
    e = float(out["energy"].item())
    fr = float(np.linalg.norm(f - ref["f"]) / np.linalg.norm(ref["f"]))
    pr = float(np.linalg.norm(phi - ref["phi"]) / np.linalg.norm(ref["phi"]))
    er = abs(e - ref["energy"]) / abs(ref["energy"])
    return {"force_rel_rms": fr, "phi_rel_rms": pr, "energy_rel": er,
            "within_bars": bool(fr <= 1e-5 and pr <= 1e-5 and er <= 1e-7)}


def cpu_leg(system, out):
    """The FP64 oracle on the timed inputs: its time on every host core (the
    CPU baseline) and the parity of the GPU outputs against it; then the
    one-thread oracle on the 1,000-atom cloud and the 24,000-atom box."""
    import oracle
    from paper_1402_7216_amd import inputs
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    ref = oracle.system_msm(system, threads=cores)
    t = time.perf_counter() - t0
    one = {}
    for name, make in (("cloud1k", inputs.cloud_1k), ("water24k", inputs.water_24k)):
        s = make()
        t1 = time.perf_counter()
        oracle.system_msm(s, threads=1)
        dt = time.perf_counter() - t1
        one[name] = {"s": round(dt, 4), "atom_evals_per_s": s.n / dt}
    base = {"value": system.n / t, "unit": "atom-evals/s", "cores": cores, "kind": "oracle",
            "sample": f"one full {system.n}-atom evaluation (energy, forces, potentials) in FP64 "
                      f"on {cores} threads, {t:.2f} s",
            "cpu_model": cpu_model(), "one_thread": one}
    return base, parity(out, ref)


TUNE_CACHE = None     # tuning cache consulted by autotune() (set in main)


def autotune(obj, x, y, z, q, trials):
    """Apply the cached tuning of a plan or batch when the cache holds its key;
    otherwise run the search (the cache is never written here)."""
    from paper_1402_7216_amd import msm
    if TUNE_CACHE and msm.cache_lookup(TUNE_CACHE, obj.tuning_key()) is not None:
        return obj.autotune(x, y, z, q, trials=trials, cache=TUNE_CACHE)
    rep = obj.autotune(x, y, z, q, trials=trials)
    rep["cache"] = "none"
    return rep


def _vs_ref(torch, out, ref):
    """Force relative RMS and energy relative difference of `out` against `ref`."""
    df = (out["f"].double() - ref["f"].double()).pow(2).sum()
    f = float(torch.sqrt(df / ref["f"].double().pow(2).sum()).item())
    e, e0 = float(out["energy"].item()), float(ref["energy"].item())
    return f, abs(e - e0) / abs(e0)


def coarse_leg(msm, torch, s, t_msm, steps, warmup, x, y, z, q, ref):
    """The cheap pair methods the thesis proposes as coarse propagators G
    (plain cutoff, shifted-force smoothed cutoff, Wolf summation, rc = a,
    Wolf alpha = 0.2 / A) on the same inputs, each autotuned over its cell
    knobs; Q_F/G = t(MSM) / t(G), the ratio the thesis estimates as about 60
    from operation counts, and each G's distance from the MSM result F."""
    res = {}
    for kind in ("cutoff", "shifted_force", "wolf"):
        plan = msm.pair_plan_for(s, kind, alpha=0.2)
        out = plan.compute(x, y, z, q)
        torch.cuda.synchronize()
        plan.check()
        autotune(plan, x, y, z, q, 10)
        mean, med = event_timed(torch, lambda: plan.compute(x, y, z, q, out=out), steps, warmup)
        plan.check()
        out = plan.compute(x, y, z, q, out=out)
        f_err, e_err = _vs_ref(torch, out, ref)
        res[kind] = {"ms": round(mean * 1e3, 5), "ms_median": round(med * 1e3, 5),
                     "atom_evals_per_s": s.n / mean, "q_f_over_g": round(t_msm / mean, 3),
                     "force_rel_rms_vs_F": round(f_err, 6), "energy_rel_vs_F": round(e_err, 6),
                     "tuning": plan.tuning()}
    return res


def cheap_msm_leg(msm, torch, workmodel, s, t_msm, work_f, steps, warmup, x, y, z, q, ref):
    """MSM itself as the coarse propagator G, on the same inputs: the finest
    grid four times coarser (h -> 4h), or the finest-grid cutoff halved
    (a = 6 A, every level's cutoff halving with it).  Reports the measured
    Q_F/G, the FLOP-model ratio of the two evaluations, and G's distance from
    F."""
    import dataclasses
    res = {}
    for name, kw in (("coarse_grid_4h", dict(spacing=4.0 * s.spacing)), ("short_cutoff_6A", dict(cutoff=6.0))):
        v = dataclasses.replace(s, **kw)
        plan = msm.plan_for(v)
        out = plan.compute(x, y, z, q)
        torch.cuda.synchronize()
        plan.check()
        autotune(plan, x, y, z, q, 10)
        mean, med = event_timed(torch, lambda: plan.compute(x, y, z, q, out=out), steps, warmup)
        plan.check()
        out = plan.compute(x, y, z, q, out=out)
        f_err, e_err = _vs_ref(torch, out, ref)
        levels, _, gn = plan.info()
        nodes = [int(v_[0]) * int(v_[1]) * int(v_[2]) for v_ in gn]
        pairs = workmodel.count_pairs_within(v.pos64(), v.cutoff)
        work = workmodel.evaluation_work(v.n, pairs, nodes, v.cutoff, v.spacing, v.order,
                                         v.split_m or v.order // 2)
        res[name] = {"cutoff": v.cutoff, "spacing": v.spacing, "levels": levels,
                     "ms": round(mean * 1e3, 5), "ms_median": round(med * 1e3, 5),
                     "q_f_over_g": round(t_msm / mean, 3),
                     "q_f_over_g_flop_model": round(work_f / work["total"], 3),
                     "force_rel_rms_vs_F": round(f_err, 6), "energy_rel_vs_F": round(e_err, 6),
                     "tuning": plan.tuning()}
    return res


def periodic_leg(msm, torch, s, t_msm, steps, warmup, x, y, z, q):
    """The same atoms in a periodic box (the box repeated in every direction):
    the spacing nearest to the free-space one that divides the box into whole
    grid periods over 5 levels, automatic levels, the top level through its
    Ewald image sum.  Timed forces evaluation (parity is tested against the
    oracle's periodic evaluation at up to 9,000 atoms), and the shifted-force
    cutoff with periodic images."""
    import dataclasses
    from paper_1402_7216_amd import inputs
    v = dataclasses.replace(s, spacing=inputs.periodic_spacing(s.box_len[0], s.spacing, 5), levels=0)
    plan = msm.plan_for(v, periodic=True)
    out = plan.compute(x, y, z, q)
    torch.cuda.synchronize()
    plan.check()
    autotune(plan, x, y, z, q, 10)
    mean, med = event_timed(torch, lambda: plan.compute(x, y, z, q, out=out), steps, warmup)
    plan.check()
    levels, _, gn = plan.info()
    d = plan.describe()
    res = {"workload": f"{v.name} periodic: {v.n} atoms, box {v.box_len[0]:.2f} A, a = {v.cutoff} A, "
                       f"h = {v.spacing:.4f} A, order {v.order}",
           "levels": levels, "ghost_nodes": d["ghost"], "grid_nodes_with_ghosts": [list(n_) for n_ in gn],
           "ms": round(mean * 1e3, 5), "ms_median": round(med * 1e3, 5),
           "atom_evals_per_s": v.n / mean, "vs_free_space_ms": round(t_msm * 1e3, 5), "tuning": plan.tuning()}
    pp = msm.pair_plan_for(v, "shifted_force", periodic=True)
    o2 = pp.compute(x, y, z, q)
    torch.cuda.synchronize()
    pp.check()
    autotune(pp, x, y, z, q, 10)
    m2, md2 = event_timed(torch, lambda: pp.compute(x, y, z, q, out=o2), steps, warmup)
    res["shifted_force_periodic_ms"] = round(m2 * 1e3, 5)
    return res


def parareal_leg(msm, torch, reps=3):
    """One parareal window on a 27,000-ion rock-salt cluster (a = 12 A, h = 2
    A, cubic): T = 8 slices of 5 velocity Verlet steps of 1 fs, fine
    propagator MSM over all slices as one batched evaluation per force call,
    coarse propagator the shifted-force cutoff; stops when no position changes
    by more than 1e-4 A.  Against the same 40 steps run sequentially with the
    single-system MSM plan."""
    from paper_1402_7216_amd import inputs
    T, steps, dt, tol = 8, 5, 1.0, 1e-4
    ions = inputs.rock_salt(30, seed=31, cutoff=12.0, grid=2.0)
    s = ions.system
    x, y, z, q = msm.to_device(s)
    pos0 = torch.stack([x, y, z]).contiguous()
    vel0 = torch.from_numpy(ions.vel).cuda().contiguous()
    im = torch.from_numpy(ions.inv_mass).cuda()
    state0 = torch.cat([pos0, vel0]).contiguous()
    plan = msm.plan_for(s)
    autotune(plan, x, y, z, q, 10)
    fine = msm.batch_for([s] * T)
    xb = torch.cat([x] * T).contiguous()
    yb, zb, qb = torch.cat([y] * T).contiguous(), torch.cat([z] * T).contiguous(), torch.cat([q] * T).contiguous()
    autotune(fine, xb, yb, zb, qb, 5)
    coarse = msm.pair_plan_for(s, "shifted_force")
    autotune(coarse, x, y, z, q, 10)

    def timed(fn):
        ts, out = [], None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return statistics.median(ts), out

    def sequential():
        p, v = pos0.clone(), vel0.clone()
        plan.vv_run(p, v, q, im, T * steps, dt, inputs.ACCEL_SCALE)
        return p
    t_seq, p_seq = timed(sequential)
    t_pr, (states, it, res) = timed(lambda: msm.parareal(fine, coarse, q, im, state0, slices=T,
                                                        steps_per_slice=steps, dt=dt,
                                                        accel_scale=inputs.ACCEL_SCALE, tol=tol))
    # one force evaluation: single system, the batch of T (per slice), the coarse function
    t_f = event_timed(torch, lambda: plan.compute(x, y, z, q), 20, 3)[0]
    t_fb = event_timed(torch, lambda: fine.compute(xb, yb, zb, qb), 20, 3)[0]
    t_g = event_timed(torch, lambda: coarse.compute(x, y, z, q), 20, 3)[0]
    err = float((states[:3, T] - p_seq).abs().max().item())
    return {"workload": f"{s.n}-ion rock-salt cluster, a = 12 A, h = 2 A, cubic; T = {T} slices x {steps} "
                        f"velocity Verlet steps of {dt} fs; G = shifted-force cutoff; tol {tol} A",
            "iterations": it, "position_changes": [round(r, 8) for r in res],
            "ms_parareal_window": round(t_pr * 1e3, 3), "ms_sequential_fine": round(t_seq * 1e3, 3),
            "max_position_error_vs_sequential_A": err,
            "ms_force_single": round(t_f * 1e3, 5),
            "ms_force_batched_per_slice": round(t_fb * 1e3 / T, 5),
            "ms_force_coarse": round(t_g * 1e3, 5),
            "q_f_over_g": round(t_f / t_g, 3)}


def water24k_leg(msm, torch, steps, warmup):
    s = make_system("water24k")
    plan = msm.plan_for(s)
    x, y, z, q = msm.to_device(s)
    out = plan.compute(x, y, z, q)
    torch.cuda.synchronize()
    plan.check()
    autotune(plan, x, y, z, q, 20)
    graph = msm.Graph(plan, x, y, z, q, out)
    modes = {"hipGraph replay": graph.launch, "eager": lambda: plan.compute(x, y, z, q, out=out)}
    res = {k: event_timed(torch, fn, steps, warmup) for k, fn in modes.items()}
    launch = min(res, key=lambda k: res[k][0])
    plan.check()
    mean, med = res[launch]
    ref = {k: v.clone() for k, v in plan.compute(x, y, z, q, out=out).items()}
    return {"workload": describe_workload(s), "atoms": s.n, "launch": launch,
            "ms_per_step": round(mean * 1e3, 5), "ms_median": round(med * 1e3, 5),
            "atom_evals_per_s": s.n / mean, "tuning": plan.tuning(),
            "coarse_propagators": coarse_leg(msm, torch, s, mean, steps, warmup, x, y, z, q, ref)}


def water100k_grad_leg(msm, torch, steps, warmup):
    """Differentiable path on the 100,000-atom box: energy-only forward, then
    the adjoint backward (dE/dr and dE/dq), as autograd would call them."""
    s = make_system("water100k")
    plan = msm.plan_for(s)
    x, y, z, q = msm.to_device(s)
    plan.compute(x, y, z, q)
    torch.cuda.synchronize()
    plan.check()
    autotune(plan, x, y, z, q, 10)
    e = torch.empty(1, dtype=torch.float64, device="cuda")
    g = torch.ones(1, dtype=torch.float64, device="cuda")
    dpos = torch.empty((3, s.n), dtype=torch.float32, device="cuda")
    dq = torch.empty(s.n, dtype=torch.float32, device="cuda")

    def fwd_bwd():
        plan.energy(x, y, z, q, out=e)
        plan.backward(x, y, z, q, g, dpos, dq)

    mean, med = event_timed(torch, fwd_bwd, steps, warmup)
    fmean, fmed = event_timed(torch, lambda: plan.compute(x, y, z, q), steps, warmup)
    plan.check()
    return {"workload": describe_workload(s), "atoms": s.n,
            "ms_forward_backward": round(mean * 1e3, 5), "ms_forward_backward_median": round(med * 1e3, 5),
            "atom_evals_per_s_forward_backward": s.n / mean,
            "ms_forces_eval": round(fmean * 1e3, 5)}


def batched_leg(msm, torch, workmodel, steps, warmup, do_tune):
    """64 uneven water replicas (2,000-60,000 atoms, a = 10 A, h = 2 A): one
    batched graph replay against 64 single-system evaluations in sequence,
    forward (energy, forces, potentials) and forward + backward (energy, then
    dE/dr and dE/dq)."""
    from paper_1402_7216_amd import inputs
    reps = inputs.water_replicas(64)
    b = msm.batch_for(reps)
    x, y, z, q = msm.batch_to_device(reps)
    out = b.compute(x, y, z, q)
    torch.cuda.synchronize()
    b.check()
    best = autotune(b, x, y, z, q, 5)["best"] if do_tune else None
    graph = b.graph(x, y, z, q, out)
    plans = [msm.plan_for(s) for s in reps]
    ins = [msm.to_device(s) for s in reps]
    outs = [p.compute(*i) for p, i in zip(plans, ins)]
    graphs = [msm.Graph(p, *i, o) for p, i, o in zip(plans, ins, outs)]
    t_batch, t_batch_med = event_timed(torch, graph.launch, steps, warmup)
    t_seq_graph, _ = event_timed(torch, lambda: [g.launch() for g in graphs], steps, warmup)
    t_seq_eager, _ = event_timed(torch, lambda: [p.compute(*i, out=o) for p, i, o in zip(plans, ins, outs)],
                                 steps, warmup)
    # forward + backward
    e = torch.empty(b.n_sys, dtype=torch.float64, device="cuda")
    gs = torch.ones(b.n_sys, dtype=torch.float64, device="cuda")
    dpos = torch.empty((3, b.n), dtype=torch.float32, device="cuda")
    dq = torch.empty(b.n, dtype=torch.float32, device="cuda")

    def batch_fb():
        e.copy_(b.energy(x, y, z, q))
        b.backward(x, y, z, q, gs, dpos, dq)

    g1 = torch.ones(1, dtype=torch.float64, device="cuda")
    grads = [(torch.empty((3, p.n), dtype=torch.float32, device="cuda"),
              torch.empty(p.n, dtype=torch.float32, device="cuda")) for p in plans]

    def seq_fb():
        for p, i, (gp, gq) in zip(plans, ins, grads):
            p.energy(*i)
            p.backward(*i, g1, gp, gq)

    t_fb, t_fb_med = event_timed(torch, batch_fb, steps, warmup)
    t_seq_fb, _ = event_timed(torch, seq_fb, steps, warmup)
    b.check()
    # whole-batch algorithmic work and its rate against the FP32 vector peak
    flop = 0.0
    for s, p in zip(reps, plans):
        _, _, gn = p.info()
        nodes = [int(v[0]) * int(v[1]) * int(v[2]) for v in gn]
        pairs = workmodel.count_pairs_within(s.pos64(), s.cutoff)
        flop += workmodel.evaluation_work(s.n, pairs, nodes, s.cutoff, s.spacing, s.order,
                                          s.split_m or s.order // 2)["total"]
    ach = flop / t_batch / 1e12
    n = b.n
    return {"workload": "64 rigid-water replicas, 2k-60k atoms each (a = 10 A, h = 2 A, cubic)",
            "atoms": n, "ms_batched_graph": round(t_batch * 1e3, 4),
            "ms_batched_graph_median": round(t_batch_med * 1e3, 4),
            "ms_64_sequential_graphs": round(t_seq_graph * 1e3, 4),
            "ms_64_sequential_eager": round(t_seq_eager * 1e3, 4),
            "atom_evals_per_s": n / t_batch,
            "speedup_vs_sequential_eager": round(t_seq_eager / t_batch, 3),
            "speedup_vs_sequential_graphs": round(t_seq_graph / t_batch, 3),
            "ms_batched_forward_backward": round(t_fb * 1e3, 4),
            "ms_batched_forward_backward_median": round(t_fb_med * 1e3, 4),
            "ms_64_sequential_forward_backward": round(t_seq_fb * 1e3, 4),
            "atom_evals_per_s_forward_backward": n / t_fb,
            "speedup_forward_backward_vs_sequential": round(t_seq_fb / t_fb, 3),
            "roofline": {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK_FP32_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_TFLOPS, 4),
                         "scope": "whole batched evaluation", "algorithmic_flop": flop},
            "tuning": best}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="water1m", choices=WORKLOADS)
    ap.add_argument("--launch", default="best", choices=("best", "hipGraph", "eager"),
                    help="launch mode to time (best: time both, report the faster)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the plan's default tuning")
    ap.add_argument("--retune", action="store_true",
                    help="run the autotuner's search even where the package's tuning cache has an entry")
    ap.add_argument("--tuning", default=None,
                    help="JSON tuning to apply instead of autotuning, e.g. the config.tuning of an "
                         "earlier run (for profiler passes over the timed configuration)")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle (CPU baseline and parity)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 24k, 100k-gradient and 64-replica legs")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 256 MiB device buffer 5 times (the reference kernel that scales the "
                         "FETCH_SIZE / WRITE_SIZE counters to bytes)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build evaluates each system on a single "
              "MI355X; run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1402_7216_amd import msm, workmodel
    global TUNE_CACHE
    TUNE_CACHE = None if args.retune or not os.path.exists(msm.TUNING_CACHE) else msm.TUNING_CACHE

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": src.numel() * 4}), flush=True)
        return
    s = make_system(args.workload)
    plan = msm.plan_for(s)
    x, y, z, q = msm.to_device(s)
    out = plan.compute(x, y, z, q)
    torch.cuda.synchronize()
    plan.check()
    levels, glo, gn = plan.info()
    nodes = [int(np.prod(v)) for v in gn]
    tuning_source = "default"
    if args.tuning:
        plan.tune(**json.loads(args.tuning))
        tuning_source = "--tuning"
    elif not args.no_autotune:
        tune_rep = autotune(plan, x, y, z, q, 40 if s.n < 200000 else 10)
        tuning_source = "cache " + plan.tuning_key() if tune_rep.get("cache") == "hit" else "search"

    graph = msm.Graph(plan, x, y, z, q, out)
    # both launch modes time the same evaluation; the faster one is reported
    modes = {"hipGraph replay": graph.launch, "eager": lambda: plan.compute(x, y, z, q, out=out)}
    if args.launch != "best":
        modes = {k: v for k, v in modes.items() if k.startswith(args.launch)}
    mode_sec = {k: event_timed(torch, fn, args.steps, args.warmup) for k, fn in modes.items()}
    launch = min(mode_sec, key=lambda k: mode_sec[k][0])
    sec, sec_med = mode_sec[launch]
    plan.check()
    # the outputs of the timed configuration (for the parity check)
    out = plan.compute(x, y, z, q, out=out)
    torch.cuda.synchronize()
    timed_out = {k: v.clone() for k, v in out.items()}

    # per-stage durations in the timed schedule: each stage's launches bracketed
    # by HIP events on the stream they run on (side streams included), over K
    # more evaluations identical to the timed ones
    def stage_pass(live, n):
        plan.profile(True, live=live)
        acc = {}
        for _ in range(n):
            plan.compute(x, y, z, q, out=out)
            for k, v in plan.stage_ms().items():
                acc[k] = acc.get(k, 0.0) + v
        plan.profile(False)
        return {k: v / n for k, v in acc.items()}

    stage_live = stage_pass(True, args.steps)
    # and each stage alone (in order on one stream): where the time goes
    stage_ms = stage_pass(False, 5)

    m = s.split_m or s.order // 2
    n_pairs = workmodel.count_pairs_within(s.pos64(), s.cutoff)
    work = workmodel.evaluation_work(s.n, n_pairs, nodes, s.cutoff, s.spacing, s.order, m)
    kernel_flops = {"short_range": work["short"], "lattice_cutoff": work["lattice"]}
    # the dominant kernel by its own (in-order) time; a side-stream stage's live
    # time also counts the compute units the other stream holds
    dom = max(kernel_flops, key=lambda k: stage_ms.get(k, 0.0))
    dom_s = stage_live[dom] * 1e-3
    achieved = kernel_flops[dom] / dom_s / 1e12
    alone = kernel_flops[dom] / (stage_ms[dom] * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "traffic": traffic_for(dom, s.name), "kernel": dom,
                "kernel_ms": round(stage_live[dom], 5), "kernel_flop": kernel_flops[dom],
                "kernel_ms_alone": round(stage_ms[dom], 5),
                "frac_alone": round(alone / PEAK_FP32_TFLOPS, 4)}

    rec = {
        "metric": "MSM atom-evals/s (E+F)",
        "value": s.n / sec,
        "unit": "atom-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "ms_per_step_median": sec_med * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": describe_workload(s), "n_atoms": s.n, "cutoff": s.cutoff,
                   "spacing": s.spacing, "order": s.order, "levels": levels,
                   "grid_sides": [int(v[0]) for v in gn], "launch": launch, "tuning": plan.tuning(),
                   "tuning_source": tuning_source},
        "ms_per_launch_mode": {k: round(v[0] * 1e3, 5) for k, v in mode_sec.items()},
        "roofline": roofline,
        "stages_ms": {k: round(v, 5) for k, v in stage_ms.items()},
        "stages_ms_live": {k: round(v, 5) for k, v in stage_live.items()},
        "algorithmic_tflops_per_step": round(work["total"] / sec / 1e12, 3),
        "algorithmic_flop_per_eval": work["total"],
        "unique_pairs": n_pairs,
    }
    if not args.no_extras:
        rec["coarse_propagators"] = coarse_leg(msm, torch, s, sec, args.steps, args.warmup, x, y, z, q,
                                               timed_out)
        rec["cheap_msm_propagators"] = cheap_msm_leg(msm, torch, workmodel, s, sec, work["total"], args.steps,
                                                     args.warmup, x, y, z, q, timed_out)
        rec["extras"] = {
            "water24k": water24k_leg(msm, torch, max(args.steps, 50), args.warmup),
            "water100k_forward_backward": water100k_grad_leg(msm, torch, max(args.steps, 50), args.warmup),
            "parareal": parareal_leg(msm, torch),
            "periodic": periodic_leg(msm, torch, s, sec, args.steps, args.warmup, x, y, z, q),
            "batched": batched_leg(msm, torch, workmodel, max(20, min(args.steps, 50)), 5,
                                   not args.no_autotune),
        }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"], rec["parity"] = cpu_leg(s, timed_out)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
