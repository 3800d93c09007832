"""Benchmark of the coupled RW-MI-DELBM step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Default workload: the 128^3 FP32 channel (walls at y = 0 / 127, periodic x
and z, tau 0.7, body force 5e-6, 20 oscillating metaballs of 8-16 control
points, 1e6 walkers released as a Gaussian pulse of sigma 4, D = 0.005,
2000 steps).  One step = one coupled step: particle poses + walker cull mask,
PSM-BGK collide-stream (writes u), walker advection/diffusion with the
near-surface queue.  Inputs are resident in HBM before the timed region.

Prints one JSON line with MLUPS (all lattice nodes per second), walker-steps
per second, the fluid kernel's achieved HBM bandwidth against the 8 TB/s peak
(algorithmic bytes over its average duration from HIP events recorded around
windows of consecutive step launches covering the timed region) and the FP64
CPU oracle timed on a bounded sample of the same workload on this host.

Other workloads (own JSON line each, not the headline):
  --workload oscillator --precision fp16|bf16|fp32|fp64   256^3 oscillator
  --workload precision                                    all storage modes vs FP64
  --workload batch                                        64-simulation sweep
  --workload copy [--lattice MiB]                         plain copy (HBM counter calibration)
  --workload serve [--rate 20 --duration 15]              Poisson request stream (disabled, see
                                                          paper_2308_05007_amd.serve.DISABLED)
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
ELEM = {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2}
UELEM = {"fp64": 8, "fp32": 4, "fp16": 4, "bf16": 4}
DTYPE = {"fp64": "f64", "fp32": "f32", "fp16": "f16-store/f32", "bf16": "bf16-store/f32"}
METRIC = "MLUPS + walker-steps/s (1 GPU, % HBM roofline); batched/served vs plain at tol"


def fluid_nodes(cfg):
    n = cfg["domain"]["n"]
    bc = cfg["domain"]["bc"]
    m = 1
    for a in range(3):
        m *= n[a] - 2 if bc[a] == "wall" else n[a]
    return m


def fluid_bytes_per_node(prec):
    """Algorithmic bytes of the collide-stream per fluid node: 19 reads and 19
    writes of the stored distribution plus the velocity the walkers need
    (3 components); the density the kernel also writes is not credited."""
    return 38 * ELEM[prec] + 3 * UELEM[prec]


def walker_bytes_per_step(prec):
    """Algorithmic bytes of one walker step: its cell index and three offsets
    read and written back.  Image counts (touched only on a periodic wrap)
    and the velocity corners (shared between walkers, served from cache) are
    not credited."""
    return 2 * (4 + 3 * (8 if prec == "fp64" else 4))


def kernel_source_hash(prec):
    """Hash of the sources the step kernel of this precision is built from."""
    h = hashlib.sha256()
    unit = "k_fp64.hip" if prec == "fp64" else "k_lowp.hip"
    for f in ("step_impl.h", "step_map.h", "lbm_impl.h", "walk_impl.h", "pro_impl.h", "dev_common.h", "launch.h",
              unit):
        with open(os.path.join(ROOT, "paper_2308_05007_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_traffic(workload_key, prec):
    """HBM bytes per full step launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "step_traffic.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    e = d.get(workload_key)
    if not e or e.get("kernel_source_sha256_16") != kernel_source_hash(prec):
        return None
    return e.get("hbm_bytes_per_launch")


def cpu_baseline(cfg, seconds=15.0, max_steps=200):
    """The FP64 oracle on this host's cores: first steps of the same workload
    (seeding excluded), as many as fit in about `seconds`."""
    import oracle
    o = oracle.build_domain(cfg)
    w = cfg["walkers"]
    o.seed(w, w["n"])
    t0 = time.perf_counter()
    steps = 0
    while steps < max_steps:
        o.step(1)
        steps += 1
        if time.perf_counter() - t0 > seconds:
            break
    dt = time.perf_counter() - t0
    N = int(np.prod(cfg["domain"]["n"]))
    cores = int(os.environ.get("OMP_NUM_THREADS") or len(os.sched_getaffinity(0)))
    return {"value": N * steps / dt / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "walker_steps_per_s": w["n"] * steps / dt,
            "sample": "FP64 oracle, first %d coupled steps of %s (%d nodes, %d walkers), %.1f s"
                      % (steps, cfg["name"], N, w["n"], dt)}


def run_plain(cfg, steps, warmup, prec, timing=8, graph=False):
    """Warm up, then time `steps` steps; HIP events on the domain stream
    bracket windows of `timing` consecutive step launches (0: none)."""
    from paper_2308_05007_amd import binding as B
    import torch
    dom = B.build_domain(cfg, device=0)
    if graph:
        dom.set("use_graph", 1)
    dom.step(warmup)
    dom.sync()
    torch.cuda.synchronize()
    if timing:
        dom.set("timing", timing)
        dom.kernel_times()  # clear
    t0 = time.perf_counter()
    dom.step(steps)
    dom.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = dom.kernel_times() if timing else {}
    mom = dom.moments()
    return dom, dt, kt, mom


def bench_plain(args):
    from paper_2308_05007_amd import workloads as W
    if args.workload == "channel":
        cfg = W.config_channel(precision=args.precision or "fp32")
        key = "channel_128_" + (args.precision or "fp32")
    else:
        cfg = W.config_oscillator(precision=args.precision or "fp16", n_walkers=args.walkers or 10_000_000)
        key = "oscillator_256_" + (args.precision or "fp16")
    prec = cfg["domain"]["precision"]
    steps, warmup = args.steps, args.warmup
    dom, dt, kt, mom = run_plain(cfg, steps, warmup, prec, timing=args.timing_every, graph=False)
    N = int(np.prod(cfg["domain"]["n"]))
    nw = cfg["walkers"]["n"]
    assert mom["n_walkers"] == nw, "walker count not conserved"
    mlups = N * steps / dt / 1e6
    ms_total, launches, fluid_launches, walker_launches = kt
    avg_s = ms_total / 1e3 / max(launches, 1)
    # a full launch carries one fluid update and one walker step
    fb, wb = fluid_nodes(cfg) * fluid_bytes_per_node(prec), nw * walker_bytes_per_step(prec)
    bytes_launch = fb + wb
    achieved = (fluid_launches * fb + walker_launches * wb) / (ms_total / 1e3) / 1e9
    traffic = pmc_traffic(key, prec)
    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": round(dt / steps * 1e3, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[prec], "data": "synthetic (seeded metaballs and walkers; no datasets)",
        "config": {"workload": key, "lattice": list(cfg["domain"]["n"]), "bc": list(cfg["domain"]["bc"]),
                   "particles": len(cfg["particles"]), "walkers": nw, "precision": prec,
                   "steps_per_run": cfg["steps"]},
        "walker_steps_per_s": round(nw * steps / dt, 1),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": "k_step (fused: PSM-BGK collide + pull-stream, walkers, particle prologue)",
                     "bytes_per_launch": bytes_launch, "avg_launch_us": round(avg_s * 1e6, 2),
                     "timed_launches": launches, "timing_window": args.timing_every},
        "counters": mom["counters"],
        "near_surface_per_step": round(mom["near_surface"] / max(mom["step"], 1), 1),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, seconds=args.cpu_seconds)
    print(json.dumps(out), flush=True)


def bench_precision(args):
    """The oscillator in every storage mode against the FP64 GPU run."""
    from paper_2308_05007_amd import precision, workloads as W
    n = args.lattice or 256
    cfg = W.config_oscillator(n=n, n_particles=args.particles or 64, n_walkers=args.walkers or 10_000_000,
                              steps=args.steps)
    rep = precision.report(cfg, steps=args.steps, every=max(1, args.steps // 100))
    print(json.dumps({"metric": "precision modes vs FP64 (velocity L2, concentration L2, D_alpha)",
                      "config": {"workload": cfg["name"].rsplit("_", 1)[0], "lattice": [n] * 3,
                                 "particles": len(cfg["particles"]), "walkers": cfg["walkers"]["n"],
                                 "steps": args.steps},
                      "report": rep}), flush=True)


def bench_copy(args):
    """Device-to-device copy of a known size through one elementwise kernel
    (y = x * 1): the reference for the HBM byte counters and the measured
    copy ceiling of this GPU."""
    import torch
    nbytes = (args.lattice or 1024) << 20  # MiB per tensor
    x = torch.rand(nbytes // 4, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    reps = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.mul(x, 1.0, out=y)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3 / reps
    print(json.dumps({"metric": "device copy (y = x * 1)", "bytes_read": nbytes, "bytes_written": nbytes,
                      "us_per_copy": round(s * 1e6, 2), "GB_per_s": round(2 * nbytes / s / 1e9, 1)}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="channel", choices=["channel", "oscillator", "precision", "batch", "serve", "copy"])
    ap.add_argument("--lattice", type=int, default=None)
    ap.add_argument("--rate", type=float, default=None)
    ap.add_argument("--duration", type=float, default=None)
    ap.add_argument("--particles", type=int, default=None)
    ap.add_argument("--precision", default=None)
    ap.add_argument("--walkers", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--timing-every", type=int, default=32,
                    help="HIP events bracket windows of this many consecutive step launches")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.workload in ("channel", "oscillator"):
        bench_plain(args)
    elif args.workload == "precision":
        bench_precision(args)
    elif args.workload == "copy":
        bench_copy(args)
    elif args.workload == "batch":
        from paper_2308_05007_amd import batchbench
        batchbench.main(args)
    else:
        from paper_2308_05007_amd import serve
        serve.bench(args)


if __name__ == "__main__":
    main()
