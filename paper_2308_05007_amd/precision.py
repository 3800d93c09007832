"""Precision modes: the same workload in FP64, FP32, FP16-storage and
BF16-storage, compared with the FP64 run.

Every mode runs the same protocol on the GPU: `steps` coupled steps with the
FP64 moments read every `every` steps.  The errors against the FP64 run are
  velocity L2       ||u - u64||_2 / ||u64||_2 over all nodes, final step
  concentration L2  ||n_s - n_s,64||_2 / ||n_s,64||_2 (Eq. 16 occupancy)
  D_alpha           relative error of the dispersion coefficient (Eq. 38-40)
  positions         distance between a walker's FP64 and low-precision
                    positions (same walker id), median / 99th percentile / max
The dispersion coefficient follows Sec. 4 (Eq. 38-40) through the library's
rwmi_dispersion_from_moments on the moment series (dispersion along z, the
particles' oscillation along x, the line fitted over the second half of the
series, 2R = 10 lattice units as in Sec. 4).
"""
import copy
import time

import numpy as np

from . import binding as B

MODES = ("fp64", "fp32", "fp16", "bf16")


def run_protocol(cfg, precision, steps=None, every=50, device=0):
    c = copy.deepcopy(cfg)
    c["domain"]["precision"] = precision
    steps = int(steps or c["steps"])
    d = B.build_domain(c, device=device)
    nw = c["walkers"]["n"]
    ser = []
    t0 = time.perf_counter()
    done = 0
    while True:
        m = d.moments()
        assert m["n_walkers"] == nw, "walker count not conserved"
        ser.append(m)
        if done >= steps:
            break
        k = min(every, steps - done)
        d.step(k)
        done += k
    wall = time.perf_counter() - t0
    u, rho = d.velocity()
    out = dict(series=ser, u=u, rho=rho, occ=d.occupancy().astype(np.float64),
               walkers=d.walkers(), counters=d.moments()["counters"], wall_s=wall, n=c["domain"]["n"],
               precision=precision, steps=steps)
    d.close()
    return out


def dispersion(res, two_r=10.0):
    """u_slip, phi, K and D_alpha of a run (Eq. 38-40, library pipeline); NaN
    where the pipeline has no answer (no slip, fewer than two samples)."""
    s = res["series"]
    N = int(np.prod(res["n"]))
    try:
        _, r = B.dispersion_from_moments(s, N, two_r, disp_axis=2, flow_axis=0, i0=len(s) // 2)
    except B.RwmiError:
        return dict(u_slip=float("nan"), phi=float("nan"), K=float("nan"), D_alpha=float("nan"))
    return dict(u_slip=r["u_slip"], phi=r["phi"], K=r["K"], D_alpha=r["D_alpha"])


def positions(res):
    cell, off, img = res["walkers"]
    n = res["n"]
    c = np.stack([cell % n[0], (cell // n[0]) % n[1], cell // (n[0] * n[1])]).astype(np.float64)
    return c + img * np.asarray(n, float)[:, None] + off


def compare(ref, other):
    du = np.linalg.norm(other["u"] - ref["u"]) / np.linalg.norm(ref["u"])
    dc = np.linalg.norm(other["occ"] - ref["occ"]) / np.linalg.norm(ref["occ"])
    a, b = dispersion(ref), dispersion(other)
    dD = abs(b["D_alpha"] - a["D_alpha"]) / abs(a["D_alpha"]) if np.isfinite(a["D_alpha"]) else float("nan")
    dist = np.sqrt(((positions(other) - positions(ref)) ** 2).sum(0))
    return dict(velocity_l2=float(du), concentration_l2=float(dc), D_alpha_rel=float(dD),
                D_alpha=b["D_alpha"], D_alpha_ref=a["D_alpha"],
                pos_median=float(np.median(dist)), pos_p99=float(np.quantile(dist, 0.99)), pos_max=float(dist.max()))


def report(cfg, steps=None, every=50, modes=MODES, device=0):
    runs = {m: run_protocol(cfg, m, steps, every, device) for m in modes}
    ref = runs["fp64"]
    out = {"workload": cfg["name"], "steps": ref["steps"], "every": every,
           "fp64": dict(dispersion(ref), wall_s=ref["wall_s"])}
    for m in modes:
        if m == "fp64":
            continue
        out[m] = dict(compare(ref, runs[m]), wall_s=runs[m]["wall_s"])
    return out
