"""Fill a tuning cache for the named workloads on the current GPU.

    python -m paper_1402_7216_amd.tune_cache --out tuning.txt

Runs the autotuner's full search (nothing is read from any cache) for the
1,000,000-, 100,000- and 24,000-atom water boxes, the cheap pair methods on
the 1M and 24k boxes, and the 64-replica batch, and stores each result under
its plan or batch key in --out (msm_tuning_cache_store).  The package's
tuning_gfx950.txt was written this way on an MI355X.
"""
from __future__ import annotations

import argparse
import json
import sys

import torch

from paper_1402_7216_amd import inputs, msm

SYSTEMS = {"water1m": (inputs.water_1m, 10), "water100k": (inputs.water_100k, 10),
           "water24k": (inputs.water_24k, 20)}
PAIR_KINDS = ("cutoff", "shifted_force", "wolf")


def tune_plan(plan, x, y, z, q, trials, out, tag):
    first = plan.compute(x, y, z, q)
    torch.cuda.synchronize()
    plan.check()
    rep = plan.autotune(x, y, z, q, trials=trials)
    key = plan.tuning_key()
    msm.cache_store(out, key, **plan.tuning())
    print(json.dumps({"workload": tag, "key": key, "best": rep["best"]}), flush=True)
    del first


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", required=True, help="cache file to add the entries to")
    ap.add_argument("--only", nargs="*", default=None, help="subset of: water1m water100k water24k batch64")
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        sys.exit("tune_cache needs a GPU")
    want = set(args.only or list(SYSTEMS) + ["batch64"])
    for name, (make, trials) in SYSTEMS.items():
        if name not in want:
            continue
        s = make()
        x, y, z, q = msm.to_device(s)
        tune_plan(msm.plan_for(s), x, y, z, q, trials, args.out, name)
        if name in ("water1m", "water24k"):
            for kind in PAIR_KINDS:
                tune_plan(msm.pair_plan_for(s, kind, alpha=0.2), x, y, z, q, trials, args.out,
                          f"{name}/{kind}")
        del x, y, z, q
        torch.cuda.empty_cache()
    if "batch64" in want:
        reps = inputs.water_replicas(64)
        b = msm.batch_for(reps)
        x, y, z, q = msm.batch_to_device(reps)
        b.compute(x, y, z, q)
        torch.cuda.synchronize()
        b.check()
        rep = b.autotune(x, y, z, q, trials=5)
        key = b.tuning_key()
        t = rep["best"]
        msm.cache_store(args.out, key, **{k: t[k] for k in msm.TUNING_KEYS})
        print(json.dumps({"workload": "batch64", "key": key, "best": t}), flush=True)


if __name__ == "__main__":
    main()
