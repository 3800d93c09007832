"""Seeded synthetic inputs for the coupled random-walk / metaball / D3Q19 step.

This module only draws inputs (lattice descriptors, metaball shapes, motions,
walker release descriptors, request traces) with numpy's PCG64.  It holds none
of the method's arithmetic and is the only code shared by the oracle-backed
tests and the GPU path: both receive the same plain arrays.

The paper's own particle shapes (reconstructed from imaging, Sec. 2.2 and
Fig. 9) and its experimental setups are not available, so shapes are seeded
random metaballs: control points uniform in a ball (or an ellipsoid of aspect
ratio a, randomly rotated), weights k_i uniform in a range.  Lattice units
throughout (dx = dt = 1).

A configuration is a dict:
  domain:    n, bc (per axis "periodic" | "wall"), wall_lo / wall_hi (3 x 3
             wall velocities, row = axis), tau, F, D, rho0, u0, seed, precision
  particles: list of {b (nc x 3 offsets, world frame), k (nc), centre,
             motion ("static" | "sinusoid" | "const_vel" | "coupled"), amp,
             period, phase (in cycles), vel}
  dem:       optional parameters of the two-way coupled particles
             (coupling_params)
  walkers:   {kind ("uniform" | "gaussian" | "band" | "explicit"), n, centre,
             sigma, band=(axis, lo, hi), ref, max_attempts}
  steps:     number of coupled steps
"""
import math

import numpy as np


def _ball(rng, n, radius):
    """n points uniform in a ball of the given radius (rejection from the cube)."""
    pts = []
    while len(pts) < n:
        p = rng.uniform(-1.0, 1.0, size=3)
        if p @ p <= 1.0:
            pts.append(p * radius)
    return np.array(pts, dtype=np.float64)


def _rotation(rng):
    """Uniform random rotation matrix (Shoemake's uniform unit quaternion)."""
    u1, u2, u3 = rng.uniform(size=3)
    a, b = math.sqrt(1 - u1), math.sqrt(u1)
    w, x, y, z = (a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2),
                  b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3))
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def metaball_shape(rng, n_ctrl, spread, k_range, aspect=1.0, rotate=False):
    """Control-point offsets (n_ctrl x 3) and weights: points uniform in an
    ellipsoid with semi-axes (s, s, aspect*s), optionally randomly rotated."""
    b = _ball(rng, n_ctrl, 1.0) * np.array([spread, spread, aspect * spread])
    if rotate:
        b = b @ _rotation(rng).T
    k = rng.uniform(k_range[0], k_range[1], size=n_ctrl)
    return np.ascontiguousarray(b), np.ascontiguousarray(k)


def bounding_radius(b, k):
    """Radius beyond which the metaball value is below 1 (max |b_i| + sqrt(sum k))."""
    return float(np.max(np.sqrt((b * b).sum(1)))) + math.sqrt(float(np.sum(k)))


def place_particles(rng, n, shapes, motion_pad, walls, tries=20000, allow_fewer=False):
    """Centres by rejection: bounding spheres widened by the motion amplitude
    plus one cell do not overlap and stay clear of wall planes.  With
    allow_fewer the shapes that find no room are dropped (the centres of the
    placed prefix are returned)."""
    centres = []
    radii = []
    for b, k in shapes:
        r = bounding_radius(b, k) + motion_pad + 1.0
        for _ in range(tries):
            c = np.array([rng.uniform(0, n[a]) for a in range(3)])
            ok = True
            for a in range(3):
                if walls[a] and not (1.0 + r <= c[a] <= n[a] - 1.0 - r):
                    ok = False
            if ok:
                for c2, r2 in zip(centres, radii):
                    d = c - c2
                    for a in range(3):
                        if not walls[a]:
                            d[a] -= n[a] * round(d[a] / n[a])
                    if d @ d < (r + r2) ** 2:
                        ok = False
                        break
            if ok:
                centres.append(c)
                radii.append(r)
                break
        else:
            if allow_fewer:
                return centres
            raise RuntimeError("could not place particle")
    return centres


def _place_one(rng, n, shapes, centres, b, k, motion_pad, tries=2000):
    """A centre for shape (b, k) in a periodic box whose widened bounding
    sphere does not overlap those of the placed shapes, or None (candidates
    drawn uniformly, the first admissible one is taken)."""
    r = bounding_radius(b, k) + motion_pad + 1.0
    L = np.asarray(n, float)
    if 2 * r >= L.min():
        return None
    cand = rng.uniform(0.0, 1.0, size=(tries, 3)) * L
    if not centres:
        return cand[0]
    C = np.asarray(centres)
    R = np.array([bounding_radius(b2, k2) + motion_pad + 1.0 for b2, k2 in shapes])
    d = cand[:, None, :] - C[None, :, :]
    d -= L * np.round(d / L)
    ok = np.all((d * d).sum(-1) >= (r + R[None, :]) ** 2, axis=1)
    idx = np.flatnonzero(ok)
    return cand[idx[0]] if idx.size else None


def _domain(n, bc, tau, F=(0, 0, 0), D=0.0, seed=0, precision="fp64", u0=(0, 0, 0), wall_lo=None,
            wall_hi=None, rho0=1.0):
    return dict(n=tuple(int(v) for v in n), bc=tuple(bc), tau=float(tau), F=tuple(float(v) for v in F),
                D=float(D), seed=int(seed), precision=precision, u0=tuple(float(v) for v in u0),
                wall_lo=np.zeros(9) if wall_lo is None else np.asarray(wall_lo, float).ravel(),
                wall_hi=np.zeros(9) if wall_hi is None else np.asarray(wall_hi, float).ravel(),
                rho0=float(rho0))


def config_plain_fp64(scale=1.0):
    """32^3 periodic, tau 0.8, body force 1e-6 along x, one static metaball of
    4 control points (k ~ U[0.5,1.5], points uniform in a ball of radius 4 at
    the centre), 1e4 walkers uniform in the fluid, D = 0.01, 200 steps, Philox
    seed 0; shapes from config seed 1."""
    rng = np.random.default_rng(1)
    b, k = metaball_shape(rng, 4, 4.0, (0.5, 1.5))
    parts = [dict(b=b, k=k, centre=np.array([16.0, 16.0, 16.0]), motion="static")]
    return dict(name="plain_fp64_32c", domain=_domain((32, 32, 32), ("periodic",) * 3, 0.8, (1e-6, 0, 0), 0.01,
                                                      seed=0, precision="fp64"),
                particles=parts, walkers=dict(kind="uniform", n=int(10000 * scale), ref=(16.0, 16.0, 16.0)),
                steps=200)


def config_channel(precision="fp32", n=128, n_walkers=1_000_000, steps=2000):
    """128^3 channel, walls at y = 0 and 127 (halfway planes at y = 1 and 127),
    periodic x and z, tau 0.7, body force 5e-6 along x; 20 metaballs with 8-16
    control points (k ~ U[0.3,1.5], spread ~ U[3,8]) oscillating along x with
    amplitude 4 and period 1000 at random phases (config seed 2); 1e6 walkers
    in a Gaussian pulse (sigma 4) at the centre, D = 0.005, 2000 steps, Philox
    seed 2."""
    rng = np.random.default_rng(2)
    shapes = []
    for _ in range(20):
        nc = int(rng.integers(8, 17))
        shapes.append(metaball_shape(rng, nc, rng.uniform(3.0, 8.0), (0.3, 1.5)))
    dims = (n, n, n)
    centres = place_particles(rng, dims, shapes, 4.0, (False, True, False))
    parts = []
    for (b, k), c in zip(shapes, centres):
        parts.append(dict(b=b, k=k, centre=c, motion="sinusoid", amp=np.array([4.0, 0, 0]), period=1000.0,
                          phase=float(rng.uniform())))
    c0 = (n / 2, n / 2, n / 2)
    return dict(name="channel_%d_%s" % (n, precision),
                domain=_domain(dims, ("periodic", "wall", "periodic"), 0.7, (5e-6, 0, 0), 0.005, seed=2,
                               precision=precision),
                particles=parts, walkers=dict(kind="gaussian", n=int(n_walkers), centre=c0, sigma=4.0, ref=c0),
                steps=int(steps))


def config_oscillator(precision="fp16", n=256, n_particles=64, n_walkers=10_000_000, steps=5000):
    """256^3 periodic oscillator box: 64 metaballs of 12 control points
    (k ~ U[0.3,1.5], spread ~ U[3,8], random orientation) oscillating along x
    with amplitude 4 and period 5000 (the oscillator of Sec. 4); tau 0.8, no
    body force; 1e7 walkers in the band z in [n/2 - 0.5, n/2 + 0.5), uniform
    in x and y (the solute band of Sec. 4); D = 0.002; 5000 steps; config
    seed 3."""
    rng = np.random.default_rng(3)
    shapes = [metaball_shape(rng, 12, rng.uniform(3.0, 8.0), (0.3, 1.5), rotate=True) for _ in range(n_particles)]
    dims = (n, n, n)
    centres = place_particles(rng, dims, shapes, 4.0, (False, False, False))
    parts = [dict(b=b, k=k, centre=c, motion="sinusoid", amp=np.array([4.0, 0, 0]), period=5000.0,
                  phase=float(rng.uniform())) for (b, k), c in zip(shapes, centres)]
    h = n / 2
    return dict(name="oscillator_%d_%s" % (n, precision),
                domain=_domain(dims, ("periodic",) * 3, 0.8, (0, 0, 0), 0.002, seed=3, precision=precision),
                particles=parts,
                walkers=dict(kind="band", n=int(n_walkers), band=(2, h - 0.5, h + 0.5), ref=(h, h, h)),
                steps=int(steps))


def config_batch_member(i, precision="fp32", steps=1000):
    """One member of the 64-simulation shape sweep (config seed 4 + i): lattice
    in {48,64,80,96}^3 periodic, 4-16 metaballs of 4-20 control points
    (spread U[1.5,3], k ~ U[0.2,0.8]) with aspect ratio U[1,4], random
    orientation, oscillating (A = 4, T = 1000) -- drawn shapes that find no
    room without overlap in a small box are dropped, keeping at least 4;
    1e5-5e5 walkers uniform in the fluid; tau 0.8; D = 0.005; Philox seed
    1000 + i."""
    rng = np.random.default_rng(4 + i)
    e = int(rng.choice([48, 64, 80, 96]))
    npart = int(rng.integers(4, 17))
    shapes = [metaball_shape(rng, int(rng.integers(4, 21)), rng.uniform(1.5, 3.0), (0.2, 0.8),
                             aspect=rng.uniform(1.0, 4.0), rotate=True) for _ in range(npart)]
    dims = (e, e, e)
    # place one by one; a shape that finds no room is scaled down by 0.7
    # (offsets x 0.7, weights x 0.49 scale the metaball exactly) up to four
    # times, then dropped
    placed, centres = [], []
    for b, k in shapes:
        for _ in range(5):
            cs = _place_one(rng, dims, placed, centres, b, k, 4.0)
            if cs is not None:
                placed.append((b, k))
                centres.append(cs)
                break
            b, k = 0.7 * b, 0.49 * k
    if len(centres) < 4:
        raise RuntimeError("sweep member %d: fewer than 4 metaballs fit" % i)
    shapes = placed
    parts = [dict(b=b, k=k, centre=c, motion="sinusoid", amp=np.array([4.0, 0, 0]), period=1000.0,
                  phase=float(rng.uniform())) for (b, k), c in zip(shapes, centres)]
    nw = int(rng.integers(100_000, 500_001))
    return dict(name="sweep_%02d" % i,
                domain=_domain(dims, ("periodic",) * 3, 0.8, (0, 0, 0), 0.005, seed=1000 + i, precision=precision),
                particles=parts, walkers=dict(kind="uniform", n=nw, ref=(e / 2, e / 2, e / 2)), steps=int(steps))


def config_batch(n_sims=64, precision="fp32", steps=1000):
    return [config_batch_member(i, precision, steps) for i in range(n_sims)]


def serving_request(rid, rng, steps_range=(500, 3000), edges=(32, 48, 64, 80, 96, 112, 128),
                    walker_range=(1e4, 1e6), particle_range=(2, 32), precisions=("fp32", "fp16")):
    """One solve request of the serving trace: edge from the size classes,
    2-32 metaballs drawn (those without room in a small box shrink, then are
    dropped), log-uniform walker count, step count, storage precision; Philox
    seed = request id."""
    e = int(rng.choice(edges))
    npart = int(rng.integers(particle_range[0], particle_range[1] + 1))
    # shapes scaled to the box so that the particles fit
    smax = max(1.5, min(5.0, e / 12.0))
    shapes = [metaball_shape(rng, int(rng.integers(4, 13)), rng.uniform(1.0, smax), (0.2, 0.8),
                             aspect=rng.uniform(1.0, 2.0), rotate=True) for _ in range(npart)]
    dims = (e, e, e)
    placed, centres = [], []
    for b, k in shapes:  # shapes without room shrink by 0.7 up to four times, then are dropped
        for _ in range(5):
            c = _place_one(rng, dims, placed, centres, b, k, 2.0, tries=400)
            if c is not None:
                placed.append((b, k))
                centres.append(c)
                break
            b, k = 0.7 * b, 0.49 * k
    parts = [dict(b=b, k=k, centre=c, motion="sinusoid", amp=np.array([2.0, 0, 0]), period=1000.0,
                  phase=float(rng.uniform())) for (b, k), c in zip(placed, centres)]
    nw = int(round(math.exp(rng.uniform(math.log(walker_range[0]), math.log(walker_range[1])))))
    steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
    prec = str(rng.choice(list(precisions)))
    return dict(name="req_%d" % rid,
                domain=_domain(dims, ("periodic",) * 3, 0.8, (0, 0, 0), 0.005, seed=rid, precision=prec),
                particles=parts, walkers=dict(kind="uniform", n=nw, ref=(e / 2, e / 2, e / 2)), steps=steps)


def serving_trace(rate=20.0, duration=600.0, seed=5, **kw):
    """Poisson arrivals at `rate` per second over `duration` seconds (trace
    seed 5): list of (arrival_time, request)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    rid = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        out.append((t, serving_request(rid, rng, **kw)))
        rid += 1
    return out


def ensemble_base_shapes(seed=6):
    """Base shapes of the shape sweep of Sec. 4, synthetic stand-ins for its
    sphere and imaged particles A-D (whose geometry is not available): a
    one-point sphere, then metaballs of growing irregularity -- two points
    (slightly elongated), four points along a line (elongated), six points
    in a plane (flattened), ten random points (irregular).  Offsets and
    weights before scaling to a common volume (config seed 6)."""
    rng = np.random.default_rng(seed)
    out = {"sphere": (np.zeros((1, 3)), np.array([1.0]))}
    out["A"] = (np.array([[-0.35, 0, 0], [0.35, 0, 0]]), np.array([0.5, 0.5]))
    out["B"] = (np.array([[x, 0, 0] for x in (-0.9, -0.3, 0.3, 0.9)]), np.array([0.22, 0.3, 0.3, 0.22]))
    ang = np.arange(6) * (2 * math.pi / 6) + rng.uniform(0, 0.3, 6)
    out["C"] = (np.stack([0.75 * np.cos(ang), 0.75 * np.sin(ang), rng.uniform(-0.05, 0.05, 6)], -1),
                rng.uniform(0.12, 0.2, 6))
    b, k = metaball_shape(rng, 10, 0.8, (0.06, 0.16), aspect=1.6, rotate=True)
    out["D"] = (b, k)
    return out


def config_ensemble_member(name, b, k, realisation, shape_index=0, R=5.0, n_particles=50, n_walkers=2_000_000,
                           steps=5000, D=0.002, precision="fp32"):
    """One realisation of the oscillator case of Sec. 4 for one particle
    shape: a periodic box of 24R x 24R x 36R lattice units, n_particles copies
    of the shape (b, k: already at its final size), each randomly rotated and
    placed without overlap, all driven by the same horizontal oscillation
    (amplitude 4, period 5000, one phase: Eq. 37 read as a displacement);
    the solute band 24R x 24R x 1 at mid-height with n_walkers walkers; tau
    0.8, diffusivity D.  Realisation r differs in placement, orientation and
    Philox seed (config seed 1000 shape_index + r)."""
    sd = 1000 * shape_index + realisation
    rng = np.random.default_rng(7000 + sd)
    dims = (int(round(24 * R)), int(round(24 * R)), int(round(36 * R)))
    shapes = [(np.ascontiguousarray(np.asarray(b, float) @ _rotation(rng).T), np.asarray(k, float))
              for _ in range(n_particles)]
    centres = place_particles(rng, dims, shapes, 4.0, (False, False, False))
    parts = [dict(b=bb, k=kk, centre=c, motion="sinusoid", amp=np.array([4.0, 0, 0]), period=5000.0, phase=0.0)
             for (bb, kk), c in zip(shapes, centres)]
    h = dims[2] / 2
    return dict(name="ensemble_%s_%d" % (name, realisation),
                domain=_domain(dims, ("periodic",) * 3, 0.8, (0, 0, 0), D, seed=100 + sd, precision=precision),
                particles=parts,
                walkers=dict(kind="band", n=int(n_walkers), band=(2, h - 0.5, h + 0.5),
                             ref=(dims[0] / 2, dims[1] / 2, h)),
                steps=int(steps))


def coupling_params(nsub=100, drive_amp=1.6e-4, drive_period=5000.0, g=(0.0, 0.0, 0.0), rho_p=2.5, kn=200.0,
                    kt=None, eta_n=None, eta_t=None, mu=0.3, Rs=0.5, coupling=1, mass_scale=None):
    """Parameters of the two-way coupled particles (Eq. 4-11).  The drive is
    Eq. 37 (4 cos(2 pi t / 5000) along x) in lattice units of the paper's
    setup (dx = 1e-3 m, dt = 2e-4 s: 4 m/s^2 is 1.6e-4), one particle update
    every 1/100 of a fluid step as in the paper's time steps; no gravity.
    The contact constants are not given in the paper: k_n is chosen so that
    a contact lasts many substeps (pi sqrt(m / k_n) > 10 steps for the
    particles here), k_t = 2/7 k_n, damping at 10% of critical for a mass
    mass_scale, friction 0.3."""
    m = 1000.0 if mass_scale is None else float(mass_scale)
    kt = 2.0 / 7.0 * kn if kt is None else kt
    eta_n = 0.2 * math.sqrt(m * kn) if eta_n is None else eta_n
    eta_t = 0.2 * math.sqrt(m * kt) if eta_t is None else eta_t
    return dict(rho_p=rho_p, g=tuple(g), drive_amp=drive_amp, drive_period=drive_period, drive_dir=(1.0, 0.0, 0.0),
                kn=kn, kt=kt, eta_n=eta_n, eta_t=eta_t, mu=mu, Rs=Rs, nsub=int(nsub), coupling=int(coupling))


def config_coupled_small(seed=3, n=(26, 22, 30), bc=("periodic", "periodic", "periodic"), n_particles=3, R=3.0,
                         n_walkers=3000, steps=40, precision="fp64", g=(0.0, 0.0, 0.0), speed=0.03, D=0.02,
                         tau=0.8, nsub=20, drive_amp=1e-3, drive_period=60.0, gap=-3.0, with_prescribed=False):
    """Small lattices of two-way coupled particles for element-by-element
    parity: seeded metaballs with sqrt(sum k) = R (2-4 control points); the
    first two on a line along x, their bounding spheres `gap` apart, launched
    towards each other at `speed`; a third (when asked for) a quarter of the
    box below them along z, launched at a random velocity; a strong, fast
    drive so that the oscillation shows within a short run; walkers in a band
    at mid-height.  With walls on z the third is launched towards the lower
    wall.  (Bounding spheres overlap by 3 by default: the surfaces are about
    a cell apart, close enough for the pair to meet although the fluid
    slows them.)"""
    rng = np.random.default_rng(seed)
    shapes = []
    for i in range(n_particles):
        nc = int(rng.integers(2, 5))
        b, k = metaball_shape(rng, nc, 0.35 * R, (0.5, 1.0))
        shapes.append((b, k * (R * R / k.sum())))
    ctr = np.array([v / 2.0 for v in n])
    r0, r1 = bounding_radius(*shapes[0]), bounding_radius(*shapes[1])
    half = 0.5 * (r0 + r1 + gap)
    centres = [ctr + np.array([-half, 0.4, 0.0]), ctr + np.array([half, 0.0, 0.0])]
    vels = [np.array([speed, 0.0, 0.0]), np.array([-speed, 0.0, 0.0])]
    if n_particles > 2:
        centres.append(ctr + np.array([0.3, -0.2, -n[2] / 4.0]))
        vels.append(np.array([0.0, 0.0, -speed]) if bc[2] == "wall" else rng.uniform(-speed, speed, 3))
    parts = [dict(b=b, k=k, centre=c, motion="coupled", vel=v) for (b, k), c, v in zip(shapes, centres, vels)]
    if with_prescribed:
        b, k = metaball_shape(rng, 2, 0.5, (0.5, 1.0))
        parts.append(dict(b=b, k=k, centre=ctr + np.array([0.0, 0.0, n[2] / 4.0]), motion="sinusoid",
                          amp=np.array([1.0, 0.0, 0.0]), period=50.0, phase=0.1))
    h = n[2] / 2.0
    return dict(name="coupled_small", domain=_domain(n, bc, tau, (0, 0, 0), D, seed=seed, precision=precision),
                particles=parts,
                dem=coupling_params(nsub=nsub, drive_amp=drive_amp, drive_period=drive_period, g=g, kn=50.0,
                                    mass_scale=100.0),
                walkers=dict(kind="band", n=n_walkers, band=(2, h - 3.0, h + 3.0), ref=tuple(ctr)),
                steps=steps)


def config_coupled_oscillator(R=5.0, n_particles=50, n_walkers=2_000_000, steps=5000, precision="fp32", seed=0,
                              shape=None, D=0.002):
    """The oscillator of Sec. 4 with two-way coupled particles: a periodic
    box of 24R x 24R x 36R, n_particles seeded metaballs of radius about R
    (or copies of `shape` = (b, k)), randomly rotated and placed without
    overlap, at rest; every particle driven by Eq. 37 (coupling_params); the
    solute band 24R x 24R x 1 at mid-height; tau 0.8."""
    rng = np.random.default_rng(8000 + seed)
    dims = (int(round(24 * R)), int(round(24 * R)), int(round(36 * R)))
    shapes = []
    for i in range(n_particles):
        if shape is None:
            b, k = metaball_shape(rng, int(rng.integers(2, 6)), 0.35 * R, (0.5, 1.0), rotate=True)
            k = k * (R * R / k.sum())
        else:
            b = np.asarray(shape[0], float) @ _rotation(rng).T
            k = np.asarray(shape[1], float)
        shapes.append((np.ascontiguousarray(b), np.ascontiguousarray(k)))
    centres = place_particles(rng, dims, shapes, 1.0, (False, False, False))
    parts = [dict(b=b, k=k, centre=c, motion="coupled", vel=np.zeros(3)) for (b, k), c in zip(shapes, centres)]
    m = 2.5 * 4.0 / 3.0 * math.pi * R ** 3
    h = dims[2] / 2
    return dict(name="coupled_oscillator_%d_%s" % (int(R), precision),
                domain=_domain(dims, ("periodic",) * 3, 0.8, (0, 0, 0), D, seed=900 + seed, precision=precision),
                particles=parts, dem=coupling_params(kn=200.0, mass_scale=m),
                walkers=dict(kind="band", n=int(n_walkers), band=(2, h - 0.5, h + 0.5),
                             ref=(dims[0] / 2, dims[1] / 2, h)),
                steps=int(steps))


def config_tiny(n=(6, 5, 7), bc=("periodic", "wall", "periodic"), n_particles=1, n_walkers=64, seed=7,
                motion="sinusoid", D=0.02, tau=0.8, F=(1e-5, 0, 0), precision="fp64", steps=5, amp=1.5,
                period=40.0, spread=1.0, walker_kind="uniform", wall_u=None, u0=(0, 0, 0)):
    """Small ragged lattices for element-by-element parity."""
    rng = np.random.default_rng(seed)
    walls = tuple(b == "wall" for b in bc)
    shapes = [metaball_shape(rng, int(rng.integers(1, 5)), spread, (0.3, 0.8)) for _ in range(n_particles)]
    parts = []
    for b, k in shapes:
        c = np.array([rng.uniform(0, n[a]) if not walls[a] else n[a] / 2.0 for a in range(3)])
        parts.append(dict(b=b, k=k, centre=c, motion=motion, amp=np.array([amp, 0.3 * amp, 0.0]), period=period,
                          phase=float(rng.uniform()), vel=np.array([0.05, 0.0, 0.02])))
    wl = np.zeros(9)
    wh = np.zeros(9)
    if wall_u is not None:
        wl[:] = np.asarray(wall_u[0], float).ravel()
        wh[:] = np.asarray(wall_u[1], float).ravel()
    c0 = tuple(v / 2 for v in n)
    return dict(name="tiny", domain=_domain(n, bc, tau, F, D, seed=seed, precision=precision, wall_lo=wl,
                                            wall_hi=wh, u0=u0),
                particles=parts, walkers=dict(kind=walker_kind, n=n_walkers, ref=c0, centre=c0, sigma=1.0),
                steps=steps)
