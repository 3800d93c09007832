"""The shape sweep of Sec. 4 (Eq. 38-45): for each particle shape, several
realisations of the oscillator case stepped together on the GPU as one
batch; their concentration profiles along z averaged over realisations and a
Gaussian fitted to the average at every read-out (rwmi_gaussian_fit), giving
the variance series of Eq. 38; U_slip from the realisation-averaged fluid and
particle velocities (Eq. 39), the solid fraction, K and D_alpha (Eq. 40,
rwmi_dispersion_fit); the shape features of Eq. 41-44 of every shape and the
Spearman correlations of Eq. 45 between them and D_alpha.

The GPU does every step of the method and the profile counts
(rwmi_read_profile); the host only averages the counts over realisations and
calls the library's fits.
"""
import json
import math
import time

import numpy as np

from . import autotune
from . import binding as B
from . import shapes as S
from . import workloads as W


def equal_volume_shapes(R=5.0, h=0.1, seed=6):
    """The base shapes, each scaled to the volume of a sphere of radius R
    (offsets x s, weights x s^2 scale a metaball exactly)."""
    out = {}
    target = 4.0 / 3.0 * math.pi * R ** 3
    for name, (b, k) in W.ensemble_base_shapes(seed).items():
        body = S.Metaball(b, k)
        # a first estimate on a grid of about 25 cells per bounding radius,
        # then one correction on the scaled body with spacing h
        s0 = (target / S.volume_area(body, body.radius / 25.0)[0]) ** (1.0 / 3.0)
        body = body.scaled(s0)
        s1 = (target / S.volume_area(body, h)[0]) ** (1.0 / 3.0)
        out[name] = body.scaled(s1)
    return out


def _fit_var(z, profile):
    """Variance of the Gaussian fitted to a profile, NaN while the band still
    occupies fewer than three layers (the fit is not determined)."""
    if np.count_nonzero(profile > 0) < 3:
        return float("nan")
    return B.gaussian_fit(z, profile)[2]


def run(shapes, realisations=4, steps=5000, every=50, R=5.0, n_particles=50, n_walkers=2_000_000, D=0.002,
        precision="fp32", two_r=None, i0_frac=0.5, use_graph=True, device=0):
    """Step every realisation of every shape as one batch; return the
    realisation-averaged series per shape and the dispersion results."""
    names = list(shapes)
    cfgs, owner = [], []
    for si, name in enumerate(names):
        body = shapes[name]
        for r in range(realisations):
            cfgs.append(W.config_ensemble_member(name, body.b, body.k, r, shape_index=si, R=R, n_particles=n_particles,
                                                 n_walkers=n_walkers, steps=steps, D=D, precision=precision))
            owner.append(name)
    doms = [B.build_domain(c, device=device) for c in cfgs]
    autotune.set_batch_streaming(doms, cfgs)
    bt = B.Batch(device=device)
    for d in doms:
        bt.add(d)
    if use_graph:
        bt.set("use_graph", 1)
    nz = cfgs[0]["domain"]["n"][2]
    ser = {n: {"t": [], "profile": [], "fluid_u": [], "particle_v": [], "solid": []} for n in names}
    done = 0
    t_gpu = 0.0
    while True:
        for n in names:
            ser[n]["profile"].append(np.zeros(nz))
            ser[n]["fluid_u"].append(np.zeros(3))
            ser[n]["particle_v"].append(np.zeros(3))
            ser[n]["solid"].append(0.0)
            ser[n]["t"].append(done)
        for d, n in zip(doms, owner):
            ser[n]["profile"][-1] += d.profile(2) / realisations
            m = d.moments()
            ser[n]["fluid_u"][-1] += m["fluid_u"] / realisations
            ser[n]["particle_v"][-1] += m["particle_v"] / realisations
            ser[n]["solid"][-1] += m["solid_volume"] / realisations
        if done >= steps:
            break
        k = min(every, steps - done)
        t0 = time.perf_counter()
        bt.step(k)
        bt.sync()
        t_gpu += time.perf_counter() - t0
        done += k
    bt.close()
    for d in doms:
        d.close()
    nodes = int(np.prod(cfgs[0]["domain"]["n"]))
    two_r = 2.0 * R if two_r is None else two_r
    z = np.arange(nz) + 0.5
    res = {}
    for n in names:
        s = ser[n]
        sig2 = np.array([_fit_var(z, p) for p in s["profile"]])
        t = np.array(s["t"], float)
        fu = np.array(s["fluid_u"])[:, 0]
        pv = np.array(s["particle_v"])[:, 0]
        u_slip = abs(float(fu.max() - pv.max()))
        sol = np.array(s["solid"])
        phi = float(sol[t > 0].mean() / nodes) if np.any(t > 0) else 0.0
        i0 = int(len(t) * i0_frac)
        if not np.all(np.isfinite(sig2[i0:])):
            raise RuntimeError("%s: a profile of the fitted window has fewer than three occupied layers" % n)
        K, Da, off = B.dispersion_fit(t, sig2, two_r, u_slip, phi, i0=i0)
        res[n] = {"t": t.tolist(), "sigma2": sig2.tolist(), "u_slip": u_slip, "phi": phi, "K": K, "D_alpha": Da,
                  "offset": off}
    total_nodes = nodes * len(cfgs)
    perf = {"members": len(cfgs), "nodes_per_member": nodes, "walkers_per_member": n_walkers, "steps": steps,
            "gpu_seconds": t_gpu, "MLUPS": total_nodes * steps / t_gpu / 1e6 if t_gpu > 0 else None,
            "walker_steps_per_s": n_walkers * len(cfgs) * steps / t_gpu if t_gpu > 0 else None}
    return res, ser, perf


def analyse(shapes, res, h=0.1, n_dirs=48):
    """Shape features per shape and the Spearman matrix of Eq. 45 over the
    features and D_alpha (the heatmap of Sec. 4)."""
    feats = {n: S.features(shapes[n], h=h, n_dirs=n_dirs) for n in shapes}
    cols = {"sphericity": [feats[n]["sphericity"] for n in shapes], "C_c": [feats[n]["C_c"] for n in shapes],
            "D_ns": [feats[n]["D_ns"] for n in shapes], "CSF": [feats[n]["CSF"] for n in shapes],
            "A_m": [feats[n]["A_m"] for n in shapes], "D_alpha": [res[n]["D_alpha"] for n in shapes]}
    return feats, S.spearman_matrix(cols)


def bench(args):
    """The shape sweep as a benchmark workload: five shapes, realisations of
    the oscillator case per shape, one batch."""
    R = getattr(args, "radius", None) or 5.0
    real = getattr(args, "realisations", None) or 4
    steps = args.steps if getattr(args, "steps_given", False) else 2000
    shapes = equal_volume_shapes(R)
    res, _, perf = run(shapes, realisations=real, steps=steps, every=max(1, steps // 40), R=R,
                       n_walkers=getattr(args, "walkers", None) or 2_000_000, precision=args.precision or "fp32")
    feats, corr = analyse(shapes, res, h=0.15, n_dirs=24)
    out = {"metric": "shape sweep of Sec. 4: D_alpha per shape and Spearman correlations (Eq. 38-45)",
           "config": {"workload": "ensemble_5shapes_x%d_%dx%dx%d" % ((real,) + tuple(int(round(v * R)) for v in (24, 24, 36))),
                      "steps": steps, "particles_per_member": 50, "precision": args.precision or "fp32"},
           "performance": perf,
           "shapes": {n: {"D_alpha": res[n]["D_alpha"], "K": res[n]["K"], "u_slip": res[n]["u_slip"],
                          "phi": res[n]["phi"],
                          **{k: feats[n][k] for k in ("sphericity", "C_c", "D_ns", "CSF", "A_m", "volume")}}
                      for n in shapes},
           "spearman": corr}
    print(json.dumps(out), flush=True)
