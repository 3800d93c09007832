"""Launch-shape autotuner for single domains and batches.

A candidate is (threads per block of the fused step launch, step launch
flags).  A mixed batch can also be tuned per size class (its members'
largest lattice edge): each class gets its own block size, the flags are
shared (tune_batch_classes).  The tuner builds scratch copies of the workload (the real
state is never stepped), times each candidate over a few coupled steps after a
warm-up, and keeps the fastest.  Results are cached per workload signature
(kind, precision, lattice size classes, walker magnitude, device name) in a
JSON file (RWMI_AUTOTUNE_CACHE, default ~/.cache/rwmi/autotune.json).  The
launch shape never changes results: every node and walker is computed the
same way under every candidate.
"""
import json
import math
import os
import time

from . import binding as B

BLOCKS = (128, 256, 512)
FLAGS = (0, 1, 2, 3)


def candidates():
    return [(bs, fl) for bs in BLOCKS for fl in FLAGS]


def _cache_path():
    return os.environ.get("RWMI_AUTOTUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "rwmi",
                                                                     "autotune.json")


def _load():
    try:
        with open(_cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(key, value):
    d = _load()
    d[key] = value
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as fh:
            json.dump(d, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def _device_name():
    try:
        import torch
        return torch.cuda.get_device_name(0).replace(" ", "_")
    except Exception:
        return "unknown"


def signature(kind, cfgs):
    classes = sorted({max(c["domain"]["n"]) for c in cfgs})
    precs = sorted({c["domain"]["precision"] for c in cfgs})
    nw = sum(c["walkers"]["n"] for c in cfgs)
    layout = "two" if batch_streaming(cfgs) == 1 else "own"
    return "%s|fused|%s|%s|n%d|w1e%d|%s|%s" % (kind, ",".join(precs), ",".join(map(str, classes)), len(cfgs),
                                           int(math.log10(max(nw, 1))), layout, _device_name())


# A domain streams its lattice in place while its 19 distributions fit in
# 384 MB (the library's default: the memory-side cache holds them).  A batch
# streams all of its members in every step, so their distributions together
# are the working set: above that size the members stream between two
# lattices instead (on the 64-simulation sweep, 2.4 GB of distributions:
# 24 955 against 23 345 MLUPS in place).
INPLACE_MAX_BYTES = 384 << 20
_STORE_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2}


def batch_streaming(cfgs):
    """Streaming layout for the members of one batch: 1 (two lattices) when
    their distributions together exceed INPLACE_MAX_BYTES, else None (each
    member keeps the layout its own size selects)."""
    total = sum(19 * int(math.prod(c["domain"]["n"])) * _STORE_BYTES[c["domain"].get("precision", "fp64")]
                for c in cfgs)
    return 1 if total > INPLACE_MAX_BYTES else None


def set_batch_streaming(doms, cfgs):
    """Apply batch_streaming to freshly built members (before the first step)."""
    mode = batch_streaming(cfgs)
    if mode is not None:
        for d in doms:
            d.set("streaming", mode)


def apply(target, cand):
    """Set a candidate on a Domain or a Batch."""
    bs, fl = cand
    target.set("block", bs)
    target.set("step_flags", fl)


def tune_domain(cfg, steps=20, warmup=10, use_cache=True):
    """Best (block, flags) for one domain configuration."""
    key = signature("domain", [cfg])
    if use_cache:
        hit = _load().get(key)
        if hit:
            return tuple(hit["best"])
    best, best_t, table = None, float("inf"), {}
    for cand in candidates():
        d = B.build_domain(cfg)
        apply(d, cand)
        d.step(warmup)
        d.sync()
        t0 = time.perf_counter()
        d.step(steps)
        d.sync()
        dt = (time.perf_counter() - t0) / steps
        d.close()
        table[str(cand)] = dt
        if dt < best_t:
            best, best_t = cand, dt
    _store(key, {"best": list(best), "us_per_step": best_t * 1e6, "table_us": {k: v * 1e6 for k, v in table.items()}})
    return best


def build_batch(cfgs, use_graph=True):
    doms = [B.build_domain(c) for c in cfgs]
    set_batch_streaming(doms, cfgs)
    bt = B.Batch()
    for d in doms:
        bt.add(d)
    if use_graph:
        bt.set("use_graph", 1)
    return bt, doms


def size_class(cfg):
    """Size class of a simulation: its largest lattice edge."""
    return int(max(cfg["domain"]["n"]))


def apply_classes(bt, doms, cfgs, shape):
    """Launch a batch with a block size per size class: shape = (dict class
    -> block, flags)."""
    blocks, flags = shape
    bt.set("member_blocks", 1)
    bt.set("step_flags", flags)
    for d, c in zip(doms, cfgs):
        d.set("block", blocks[str(size_class(c))])


def _time_batch(bt, steps, warmup, reps=2):
    """Seconds per step of a batch: the fastest of `reps` windows of `steps`
    steps after `warmup`.  Walkers are regrouped every 128 steps, which adds
    a few milliseconds to the window it falls in; two windows shorter than
    half that interval cannot both hold one, so the minimum is free of it."""
    bt.step(warmup)
    bt.sync()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        bt.step(steps)
        bt.sync()
        best = min(best, (time.perf_counter() - t0) / steps)
    return best


def tune_batch_classes(cfgs, steps=16, warmup=8, use_cache=True, passes=1):
    """Block size per size class, then the step flags, for a mixed batch: one
    class at a time, its members' block size is varied with the others held,
    and the batch is timed (coordinate descent over the classes, `passes`
    sweeps); the flags are chosen last for the whole batch.  Returns
    ({class: block}, flags) with classes as strings (JSON keys)."""
    key = signature("batch-classes", cfgs)
    if use_cache:
        hit = _load().get(key)
        if hit:
            return {k: int(v) for k, v in hit["blocks"].items()}, int(hit["flags"])
    classes = sorted({size_class(c) for c in cfgs})
    blocks = {str(k): 256 for k in classes}
    flags = 1
    bt, doms = build_batch(cfgs, use_graph=False)
    table = {}
    best_t = float("inf")
    for _ in range(passes):
        for k in classes:
            best_b = blocks[str(k)]
            for bs in BLOCKS:
                blocks[str(k)] = bs
                apply_classes(bt, doms, cfgs, (blocks, flags))
                dt = _time_batch(bt, steps, warmup)
                table["class %d block %d" % (k, bs)] = dt * 1e6
                if dt < best_t:
                    best_t, best_b = dt, bs
            blocks[str(k)] = best_b
    best_f = flags
    for fl in FLAGS:
        apply_classes(bt, doms, cfgs, (blocks, fl))
        dt = _time_batch(bt, steps, warmup)
        table["flags %d" % fl] = dt * 1e6
        if dt < best_t:
            best_t, best_f = dt, fl
    flags = best_f
    bt.close()
    for d in doms:
        d.close()
    _store(key, {"blocks": blocks, "flags": flags, "us_per_step": best_t * 1e6, "table_us": table})
    return blocks, flags


def tune_batch(cfgs, steps=16, warmup=8, use_cache=True, cands=None):
    """Best (block, flags) for a batch of configurations."""
    key = signature("batch", cfgs)
    if use_cache:
        hit = _load().get(key)
        if hit:
            return tuple(hit["best"])
    bt, doms = build_batch(cfgs, use_graph=False)
    best, best_t, table = None, float("inf"), {}
    for cand in cands or candidates():
        apply(bt, cand)
        dt = _time_batch(bt, steps, warmup)
        table[str(cand)] = dt
        if dt < best_t:
            best, best_t = cand, dt
    bt.close()
    for d in doms:
        d.close()
    _store(key, {"best": list(best), "us_per_step": best_t * 1e6, "table_us": {k: v * 1e6 for k, v in table.items()}})
    return best
