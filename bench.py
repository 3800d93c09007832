"""Benchmark of the coupled RW-MI-DELBM step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Default workload (the headline): the 256^3 periodic oscillator in FP32
storage -- 64 metaballs of 12 control points (random orientation) in a
prescribed sinusoidal oscillation (amplitude 4, period 5000), 1e7 walkers
released in the band z in [127.5, 128.5), D = 0.002, tau = 0.8.  Its two
lattices (2.6 GB) and velocity field stream from HBM; nothing of it fits the
256 MB memory-side cache.  One step = one coupled step: particle poses and
walker cull mask, PSM-BGK collide-stream (writes u), walker advection /
diffusion with the near-surface queue.  Inputs are resident in HBM before
the timed region.

The timed window sits mid-run: half of the workload's steps are advanced
untimed first (see burnin_steps), then W warm-up steps, then K timed steps.

Prints one JSON line: MLUPS (all lattice nodes per second), walker-steps per
second, the step kernel's achieved bandwidth in algorithmic bytes against
the 8 TB/s HBM peak (HIP events recorded around windows of consecutive step
launches that cover the timed region), the same workload with FP16 and BF16
storage, with the paper's interpolated bounce-back coupling, the 128^3 FP32
channel (whose lattice is cache-resident) and the Sec. 4 oscillator with
two-way coupled particles (both couplings) as secondary figures, and the
FP64 CPU oracle timed on a bounded sample of the headline workload on this
host, on all threads and on one.

Other workloads (own JSON line each, not the headline):
  --workload oscillator --precision fp16|bf16|fp32|fp64   256^3 oscillator alone
  --workload channel [--precision ...]                    128^3 channel alone
  --workload precision                                    all storage modes vs FP64
  --workload batch                                        64-simulation sweep
  --workload ensemble [--realisations 4 --radius 5]       shape sweep of Sec. 4 (D_alpha, Spearman)
  --workload coupled [--radius 5 --precision fp32]        Sec. 4 oscillator, two-way coupled particles
  --coupling ibb                                          interpolated bounce-back (Eq. 23-27) instead of
                                                          partially saturated cells
  --workload copy [--lattice MiB]                         plain copy (HBM counter calibration)
  --workload streams                                      the update's memory pattern without arithmetic
                                                          (1-19 read + write streams, planes and tiles)
  --workload serve [--rate 20 --duration 15]              Poisson request stream
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
    """HBM bytes per timed step launch (FETCH_SIZE and WRITE_SIZE, calibrated
    on a plain copy) and the algorithmic bytes of the same launches, from the
    committed rocprofv3 counter summary, if it was taken on the current
    kernel source; else (None, None)."""
    path = os.path.join(ROOT, "profiles", "step_traffic.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None, None
    e = d.get(workload_key)
    if not e or e.get("kernel_source_sha256_16") != kernel_source_hash(prec):
        return None, None
    return e.get("hbm_bytes_per_launch"), e.get("algorithmic_bytes_per_launch")


def _traffic_keys(workload_key, prec):
    """HBM traffic of a secondary workload's step launch from the committed
    counter summary (as for the headline), when there is one for the current
    kernel source."""
    traffic, alg = pmc_traffic(workload_key, prec)
    if not traffic or not alg:
        return {}
    return {"traffic": traffic, "traffic_over_algorithmic": round(traffic / alg, 4)}


def _oracle_sample(cfg, seconds, max_steps, threads):
    """Steps of the FP64 oracle on the workload (seeding excluded) with the
    given number of threads: at least one, then as many as fit in `seconds`."""
    import oracle
    oracle.set_threads(threads)
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
    del o
    return steps, dt


def cpu_baseline(cfg, seconds=12.0, max_steps=200, single_thread=True):
    """The FP64 oracle on this host's cores, on a bounded sample of the same
    workload: its first steps on all threads (about `seconds`), then its
    first step on one thread."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    N = int(np.prod(cfg["domain"]["n"]))
    nw = cfg["walkers"]["n"]
    steps, dt = _oracle_sample(cfg, seconds, max_steps, cores)
    out = {"value": round(N * steps / dt / 1e6, 2), "unit": "MLUPS", "cores": cores, "kind": "oracle",
           "walker_steps_per_s": round(nw * steps / dt, 1),
           "sample": "FP64 oracle, first %d coupled steps of %s (%d nodes, %d walkers) on %d threads, %.1f s"
                     % (steps, cfg["name"], N, nw, cores, dt)}
    if single_thread:
        s1, d1 = _oracle_sample(cfg, 0.0, 1, 1)
        out["single_thread"] = {"value": round(N * s1 / d1 / 1e6, 3), "unit": "MLUPS", "cores": 1,
                                "walker_steps_per_s": round(nw * s1 / d1, 1),
                                "sample": "first %d coupled step on 1 thread, %.1f s" % (s1, d1)}
    oracle.set_threads(cores)
    return out


def run_plain(cfg, steps, warmup, timing=32, graph=False, burnin=0):
    """Advance `burnin` steps (untimed: the state at mid-run), warm up, then
    time `steps` steps; HIP events on the domain stream bracket windows of
    `timing` consecutive step launches (0: none)."""
    from paper_2308_05007_amd import binding as B
    import torch
    dom = B.build_domain(cfg, device=0)
    if graph:
        dom.set("use_graph", 1)
    if burnin:
        dom.step(burnin)
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
    dom.close()
    del dom
    torch.cuda.empty_cache()
    return dt, kt, mom


def burnin_steps(cfg, args):
    """Untimed steps before the warm-up: half of the workload's run, so that
    the timed window sits mid-run.  The particles stir a fluid that starts at
    rest, and a launch takes longer as the stored values fill with nonzero
    data (the 256^3 FP32 oscillator: 537 us per launch at step 5, 598 at step
    100, 620-633 from step 1000 to 5000)."""
    return cfg["steps"] // 2 if args.burnin is None else args.burnin


def measure(cfg, key, steps, warmup, timing, burnin=0):
    """MLUPS, walker-steps/s and the step kernel's achieved bandwidth in
    algorithmic bytes for one workload."""
    prec = cfg["domain"]["precision"]
    dt, kt, mom = run_plain(cfg, steps, warmup, timing=timing, burnin=burnin)
    N = int(np.prod(cfg["domain"]["n"]))
    nw = cfg["walkers"]["n"]
    assert mom["n_walkers"] == nw, "walker count not conserved"
    ms_total, launches, fluid_launches, walker_launches = kt
    avg_s = ms_total / 1e3 / max(launches, 1)
    # a full launch carries one fluid update and one walker step
    fb, wb = fluid_nodes(cfg) * fluid_bytes_per_node(prec), nw * walker_bytes_per_step(prec)
    achieved = (fluid_launches * fb + walker_launches * wb) / (ms_total / 1e3) / 1e9
    return {"key": key, "prec": prec, "N": N, "nw": nw, "dt": dt, "steps": steps, "burnin": burnin,
            "mlups": N * steps / dt / 1e6, "wsps": nw * steps / dt, "achieved": achieved,
            "bytes_launch": fb + wb, "avg_us": avg_s * 1e6, "launches": launches, "mom": mom}


def bench_plain(args):
    from paper_2308_05007_amd import workloads as W
    headline = args.workload == "oscillator"
    prec = args.precision or "fp32"
    if headline:
        cfg = W.config_oscillator(precision=prec, n_walkers=args.walkers or 10_000_000)
        key = "oscillator_256_" + prec
    else:
        cfg = W.config_channel(precision=prec)
        key = "channel_128_" + prec
    if args.coupling == "ibb":
        cfg["domain"]["coupling"] = "ibb"
        key += "_ibb"
    if args.components != "all":
        # the same lattice and run without the walkers and/or the particles:
        # the split of the step's time and counters among its parts
        if "walkers" not in args.components:
            cfg["walkers"]["n"] = 0
        if "particles" not in args.components:
            cfg["particles"] = []
        key += "_" + args.components.replace("+", "_")
    steps, warmup = args.steps, args.warmup
    r = measure(cfg, key, steps, warmup, args.timing_every, burnin=burnin_steps(cfg, args))
    mom = r["mom"]
    traffic, traffic_alg = pmc_traffic(key, prec)
    out = {
        "metric": METRIC, "value": round(r["mlups"], 1), "unit": "MLUPS", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": round(r["dt"] / steps * 1e3, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[prec],
        "data": "synthetic (seeded metaballs and walkers; no datasets)",
        "config": {"workload": key, "lattice": list(cfg["domain"]["n"]), "bc": list(cfg["domain"]["bc"]),
                   "particles": len(cfg["particles"]), "walkers": r["nw"], "precision": prec,
                   "steps_per_run": cfg["steps"], "timed_from_step": r["burnin"] + warmup},
        "walker_steps_per_s": round(r["wsps"], 1),
        "roofline": {"bound": "hbm", "achieved": round(r["achieved"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(r["achieved"] / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "traffic_over_algorithmic": round(traffic / traffic_alg, 4) if traffic and traffic_alg else None,
                     "kernel": "k_step (fused: PSM-BGK collide + pull-stream, walkers, particle prologue)",
                     "bytes_per_launch": r["bytes_launch"], "avg_launch_us": round(r["avg_us"], 2),
                     "timed_launches": r["launches"], "timing_window": args.timing_every},
        "counters": mom["counters"],
        "near_surface_per_step": round(mom["near_surface"] / max(mom["step"], 1), 1),
    }
    if headline and prec == "fp32" and not args.no_secondary:
        sec = {}
        s2, w2 = 64, 8
        for p2 in ("fp16", "bf16"):
            c2 = W.config_oscillator(precision=p2, n_walkers=args.walkers or 10_000_000)
            q = measure(c2, "oscillator_256_" + p2, s2, w2, args.timing_every, burnin=burnin_steps(c2, args))
            sec[q["key"]] = {"MLUPS": round(q["mlups"], 1), "walker_steps_per_s": round(q["wsps"], 1),
                             **_traffic_keys(q["key"], p2),
                             "ms_per_step": round(q["dt"] / s2 * 1e3, 5), "roofline_frac": round(q["achieved"] / HBM_PEAK_GBS, 4),
                             "bytes_per_launch": q["bytes_launch"], "avg_launch_us": round(q["avg_us"], 2),
                             "steps": s2, "warmup": w2, "timed_from_step": q["burnin"] + w2}
        c3 = W.config_channel(precision="fp32")
        q = measure(c3, "channel_128_fp32", 256, 16, args.timing_every, burnin=burnin_steps(c3, args))
        sec["channel_128_fp32_cache_resident"] = {
            "MLUPS": round(q["mlups"], 1), "walker_steps_per_s": round(q["wsps"], 1),
            "ms_per_step": round(q["dt"] / 256 * 1e3, 5), "roofline_frac": round(q["achieved"] / HBM_PEAK_GBS, 4),
            "bytes_per_launch": q["bytes_launch"], "avg_launch_us": round(q["avg_us"], 2), "steps": 256, "warmup": 16,
            "timed_from_step": q["burnin"] + 16,
            "note": "the in-place lattice and velocity (160 MB + 48 MB) fit the 256 MB memory-side cache: not an HBM figure"}
        # the paper's own coupling (interpolated bounce-back, Eq. 23-27) on the same workload
        c4 = W.config_oscillator(precision="fp32", n_walkers=args.walkers or 10_000_000)
        c4["domain"]["coupling"] = "ibb"
        q = measure(c4, "oscillator_256_fp32_ibb", s2, w2, args.timing_every, burnin=burnin_steps(c4, args))
        sec[q["key"]] = {"MLUPS": round(q["mlups"], 1), "walker_steps_per_s": round(q["wsps"], 1),
                         **_traffic_keys(q["key"], "fp32"),
                         "ms_per_step": round(q["dt"] / s2 * 1e3, 5), "roofline_frac": round(q["achieved"] / HBM_PEAK_GBS, 4),
                         "bytes_per_launch": q["bytes_launch"], "avg_launch_us": round(q["avg_us"], 2),
                         "steps": s2, "warmup": w2, "timed_from_step": q["burnin"] + w2,
                         "note": "interpolated bounce-back instead of partially saturated cells; bytes credited "
                                 "as for the headline (the density and status byte it also writes are not)"}
        # two-way coupled particles (Eq. 4-11), both couplings
        for cp in ("psm", "ibb"):
            r = coupled_figures("fp32", 5.0, 2_000_000, 100, 5, 200, coupling=cp, timed_steps=16)
            sec[r["key"]] = {"MLUPS": round(r["mlups"], 1), "walker_steps_per_s": round(r["wsps"], 1),
                             "ms_per_step": round(r["dt"] / r["steps"] * 1e3, 5),
                             "roofline_frac_step_launch": round(r["achieved"] / HBM_PEAK_GBS, 4),
                             "per_launch_us": r["per_launch_us"], "steps": r["steps"], "warmup": 5,
                             "timed_from_step": r["timed_from_step"], "particles": len(r["cfg"]["particles"]),
                             "lattice": list(r["cfg"]["domain"]["n"]), "substeps": r["cfg"]["dem"]["nsub"]}
        out["secondary"] = sec
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, seconds=args.cpu_seconds)
    print(json.dumps(out), flush=True)


def coupled_figures(prec, R, n_walkers, steps, warmup, burnin, coupling="psm", timed_steps=32):
    """The oscillator of Sec. 4 with two-way coupled particles (Eq. 4-11): 50
    metaballs of radius R driven by Eq. 37 in a 24R x 24R x 36R box, walkers
    in the band.  Wall clock over `steps` steps through captured graphs
    (MLUPS); then `timed_steps` steps with every launch timed on its own: the
    fused step launch (fluid with the force sums, walkers), the particle
    update and the prologue of the masks."""
    from paper_2308_05007_amd import binding as B, workloads as W
    import torch
    cfg = W.config_coupled_oscillator(R=R, precision=prec, n_walkers=n_walkers)
    if coupling == "ibb":
        cfg["domain"]["coupling"] = "ibb"
    dom = B.build_domain(cfg, device=0)
    dom.set("use_graph", 1)
    dom.step(burnin + warmup)
    dom.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dom.step(steps)
    dom.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    dom.set("use_graph", 0)
    dom.set("timing", 1)
    dom.kernel_times()
    dom.coupling_times()
    dom.step(timed_steps)
    dom.sync()
    (ms_upd, n_upd), (ms_pro, n_pro) = dom.coupling_times()
    ms_step, launches, fl, wl = dom.kernel_times()
    mom = dom.moments()
    vmax = max(float(np.abs(dom.particle_state(p)["v"]).max()) for p in range(len(cfg["particles"])))
    dom.close()
    N = int(np.prod(cfg["domain"]["n"]))
    nw = cfg["walkers"]["n"]
    fb, wb = fluid_nodes(cfg) * fluid_bytes_per_node(prec), nw * walker_bytes_per_step(prec)
    achieved = (fl * fb + wl * wb) / (ms_step / 1e3) / 1e9
    key = "coupled_oscillator_%d_%s%s" % (int(R), prec, "_ibb" if coupling == "ibb" else "")
    return {"key": key, "cfg": cfg, "N": N, "nw": nw, "dt": dt, "steps": steps, "mlups": N * steps / dt / 1e6,
            "wsps": nw * steps / dt, "achieved": achieved, "bytes_launch": fb + wb,
            "per_launch_us": {"step (fluid + force sums, walkers)": round(ms_step * 1e3 / max(launches, 1), 2),
                              "particle update": round(ms_upd * 1e3 / max(n_upd, 1), 2),
                              "prologue (masks)": round(ms_pro * 1e3 / max(n_pro, 1), 2),
                              "timed_steps": timed_steps},
            "timed_from_step": burnin + warmup, "vmax": vmax, "mom": mom}


def bench_coupled(args):
    """One JSON line for the coupled oscillator (coupled_figures)."""
    prec = args.precision or "fp32"
    burnin = 500 if args.burnin is None else args.burnin
    r = coupled_figures(prec, args.radius or 5.0, args.walkers or 2_000_000, args.steps, args.warmup, burnin,
                        coupling=args.coupling)
    cfg, mom = r["cfg"], r["mom"]
    out = {"metric": METRIC, "value": round(r["mlups"], 1), "unit": "MLUPS", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(r["dt"] / args.steps * 1e3, 5),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[prec],
           "data": "synthetic (seeded metaballs and walkers; no datasets)",
           "config": {"workload": r["key"], "lattice": list(cfg["domain"]["n"]), "particles": len(cfg["particles"]),
                      "walkers": r["nw"], "precision": prec, "substeps": cfg["dem"]["nsub"],
                      "coupling": args.coupling, "timed_from_step": r["timed_from_step"]},
           "walker_steps_per_s": round(r["wsps"], 1),
           "per_launch_us": r["per_launch_us"],
           "roofline": {"bound": "hbm", "achieved": round(r["achieved"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(r["achieved"] / HBM_PEAK_GBS, 4), "traffic": None,
                        "kernel": "k_step with coupled particles (fluid with force sums, walkers)",
                        "bytes_per_launch": r["bytes_launch"]},
           "max_particle_speed": r["vmax"], "contact_misses": mom["contact_misses"], "counters": mom["counters"]}
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


def bench_streams(args):
    """The lattice update's memory pattern without its arithmetic or
    neighbour shifts (rwmi_stream_probe): 1, 2, 4, 8 and 19 read and as many
    write streams of 2^24 floats each (one 256^3 lattice's node count), as
    planes and in tiles of 256 nodes, and 4, 8 and 19 streams of halves in
    tiles (the 16-bit storage modes), 20 timed launches each.  The 1- and
    2-stream float cases (64 and 128 MB each way) fit the memory-side
    cache."""
    import torch
    from paper_2308_05007_amd import binding as B
    B.lib()
    n = 1 << 24
    src32 = torch.rand(19 * n, device="cuda")
    dst32 = torch.empty_like(src32)
    s = torch.cuda.current_stream()
    out = {}
    cases = [(st, t, 4) for st in (1, 2, 4, 8, 19) for t in (0, 1)] + [(st, 1, 2) for st in (4, 8, 19)]
    src16 = dst16 = None
    for streams, tiled, elem in cases:
        if elem == 2 and src16 is None:
            src16, dst16 = src32.half(), torch.empty_like(src32, dtype=torch.float16)
        src, dst = (src32, dst32) if elem == 4 else (src16, dst16)
        a, b = src[:streams * n], dst[:streams * n]
        for _ in range(3):
            B.stream_probe(streams, tiled, a, b, s)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(20):
            B.stream_probe(streams, tiled, a, b, s)
        e1.record(s)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / 20
        key = "%d_%s" % (streams, "tiled" if tiled else "planes") + ("" if elem == 4 else "_16bit")
        out[key] = {"us_per_launch": round(us, 2), "bytes": 2 * elem * streams * n,
                    "GB_per_s": round(2 * elem * streams * n / us / 1e3, 1)}
    print(json.dumps({"metric": "stream pattern bandwidth (reads + writes of 2^24 elements per stream)",
                      "unit": "GB/s", "peak": HBM_PEAK_GBS, "results": out}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="oscillator",
                    choices=["oscillator", "channel", "precision", "batch", "ensemble", "coupled", "serve", "copy",
                             "streams"])
    ap.add_argument("--lattice", type=int, default=None)
    ap.add_argument("--rate", type=float, default=None)
    ap.add_argument("--duration", type=float, default=None)
    ap.add_argument("--particles", type=int, default=None)
    ap.add_argument("--precision", default=None)
    ap.add_argument("--walkers", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="skip the FP16/BF16 and channel figures")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--realisations", type=int, default=None, help="ensemble: realisations per shape")
    ap.add_argument("--radius", type=float, default=None, help="ensemble: particle radius R in lattice units")
    ap.add_argument("--burnin", type=int, default=None,
                    help="untimed steps before the warm-up (default: half of the workload's run)")
    ap.add_argument("--components", default="all", choices=["all", "fluid", "fluid+particles", "fluid+walkers"],
                    help="oscillator/channel: run without the walkers and/or the particles (a split of the step)")
    ap.add_argument("--coupling", default="psm", choices=["psm", "ibb"],
                    help="fluid-particle coupling: partially saturated cells or interpolated bounce-back")
    ap.add_argument("--timing-every", type=int, default=32,
                    help="HIP events bracket windows of this many consecutive step launches")
    args = ap.parse_args()
    args.steps_given = any(a == "--steps" or a.startswith("--steps=") for a in sys.argv[1:])
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.workload in ("channel", "oscillator"):
        bench_plain(args)
    elif args.workload == "precision":
        bench_precision(args)
    elif args.workload == "copy":
        bench_copy(args)
    elif args.workload == "streams":
        bench_streams(args)
    elif args.workload == "batch":
        from paper_2308_05007_amd import batchbench
        batchbench.main(args)
    elif args.workload == "coupled":
        bench_coupled(args)
    elif args.workload == "ensemble":
        from paper_2308_05007_amd import ensemble
        ensemble.bench(args)
    else:
        from paper_2308_05007_amd import serve
        serve.bench(args)


if __name__ == "__main__":
    main()
