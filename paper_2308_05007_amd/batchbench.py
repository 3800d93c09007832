"""The 64-simulation shape sweep: plain one-at-a-time runs against one batch.

Plain: each simulation is created, run for its steps and read back alone
(one domain, its own launches), one after the other.  Batched: all of them in
one rwmi batch (one launch per kernel per step over every member, replayed
from a hipGraph), once with one autotuned launch shape for the whole batch
and once with an autotuned block size per size class.  Both report aggregate
node updates and walker steps per second; a few members are checked to be
bit-identical between the two paths.
"""
import json
import time

import numpy as np

from . import autotune
from . import binding as B
from . import workloads as W


def _snapshot(d):
    u, rho = d.velocity()
    cell, off, img = d.walkers()
    return u, rho, cell, off, img


def run(n_sims=64, steps=1000, precision="fp32", check=4, tune=True):
    cfgs = W.config_batch(n_sims, precision=precision, steps=steps)
    nodes = sum(int(np.prod(c["domain"]["n"])) for c in cfgs)
    walkers = sum(c["walkers"]["n"] for c in cfgs)
    cand = autotune.tune_batch(cfgs) if tune else (256, 1)
    shape = autotune.tune_batch_classes(cfgs) if tune else ({str(autotune.size_class(c)): 256 for c in cfgs}, 1)
    # plain path: one simulation at a time
    ref = {}
    t_plain = 0.0
    for i, c in enumerate(cfgs):
        d = B.build_domain(c)
        d.sync()
        t0 = time.perf_counter()
        d.step(steps)
        d.sync()
        t_plain += time.perf_counter() - t0
        if i < check:
            ref[i] = _snapshot(d)
        d.close()
    # batched paths: one launch shape for the whole batch, and one per size class
    out = {}
    same = True
    for name, setup in (("batched_one_shape", lambda bt, doms: autotune.apply(bt, cand)),
                        ("batched", lambda bt, doms: autotune.apply_classes(bt, doms, cfgs, shape))):
        bt, doms = autotune.build_batch(cfgs, use_graph=True)
        setup(bt, doms)
        bt.sync()
        t0 = time.perf_counter()
        bt.step(steps)
        bt.sync()
        t = time.perf_counter() - t0
        same &= all(all(np.array_equal(a, b) for a, b in zip(ref[i], _snapshot(doms[i]))) for i in ref)
        bt.close()
        for d in doms:
            d.close()
        out[name] = {"seconds": t, "MLUPS": nodes * steps / t / 1e6, "walker_steps_per_s": walkers * steps / t}
    return {
        "n_sims": n_sims, "steps": steps, "precision": precision, "nodes": nodes, "walkers": walkers,
        "launch_one_shape": {"block": cand[0], "step_flags": cand[1]},
        "launch_per_class": {"blocks": shape[0], "step_flags": shape[1]},
        "plain": {"seconds": t_plain, "MLUPS": nodes * steps / t_plain / 1e6,
                  "walker_steps_per_s": walkers * steps / t_plain},
        **out,
        "speedup": t_plain / out["batched"]["seconds"], "checked_members_bit_identical": bool(same),
        "checked_members": len(ref),
    }


def main(args):
    steps = args.steps if args.steps_given else 1000
    r = run(steps=steps, precision=args.precision or "fp32")
    print(json.dumps({"metric": "batched vs plain (64-simulation sweep)", "unit": "MLUPS",
                      "value": round(r["batched"]["MLUPS"], 1), "config": {"workload": "sweep_64x(48-96)^3"},
                      "report": r}), flush=True)
