"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

FP64 mode: walker counts, cells, image counts, occupancy and event counters
must match exactly.  The kernels follow the oracle's operation order with
contraction off, so velocities, densities, distributions and walker offsets
must match bit for bit as well (stricter than the 1e-10 relative the FP64
contract allows); a failure reports how many elements differ and by how
much.  The FP64 moments are sums the GPU takes in fixed chunks and the
oracle sequentially: they must agree within the error bound of recursive
summation, gamma_k times the sum of the absolute values of their terms
(_sum_close)."""
import numpy as np
import pytest

from paper_2308_05007_amd import workloads as W

pytestmark = pytest.mark.gpu

@pytest.fixture(scope="module")
def B():
    from paper_2308_05007_amd import binding
    binding.lib()
    return binding


def _pair(orc, B, cfg, seed=True):
    o = orc.build_domain(cfg)
    g = B.build_domain(cfg, seed_walkers=False)
    w = cfg.get("walkers")
    if seed and w and w.get("n", 0):
        no = o.seed(w, w["n"])
        ng = g.seed(w, w["n"], check=False)
        assert no == ng
    return o, g


def _same(a, b, what):
    """Bitwise equality of two FP64 arrays (NaNs compare equal)."""
    a = np.asarray(a)
    b = np.asarray(b)
    assert a.shape == b.shape, what
    if not np.array_equal(a, b, equal_nan=True):
        d = np.abs(a - b)
        raise AssertionError("%s: %d of %d elements differ, max diff %.3e (max |ref| %.3e)" % (
            what, int(np.count_nonzero(a != b)), a.size, float(np.nanmax(d)), float(np.max(np.abs(b)))))


def _sum_close(got, ref, abs_sum, n_terms, what, ratio=False):
    """A sum of n_terms FP64 terms that the oracle adds one after another and
    the GPU in chunks of 4096 (then the chunk partials in order): each result
    is within gamma_k sum |x_i| of the exact sum, gamma_k = k u / (1 - k u),
    u = 2^-53, k the longest chain of additions (n_terms for the oracle, at
    most 4096 + n_terms / 4096 for the GPU); a ratio of two such sums with a
    positive denominator (the fluid and particle averages) at most twice
    that, relative to the ratio's |numerator terms| / denominator."""
    got, ref, abs_sum = (np.atleast_1d(np.asarray(v, float)) for v in (got, ref, abs_sum))
    k = n_terms + 4096 + n_terms / 4096.0 + 2
    gamma = k * 2.0 ** -53 / (1 - k * 2.0 ** -53)
    bound = (2.0 if ratio else 1.0) * gamma * abs_sum
    err = np.abs(got - ref)
    assert np.all(err <= bound), "%s: diff %s, bound %s" % (what, err, bound)


def _moment_scales(o):
    """Sums of the absolute values of the terms of every FP64 moment, from the
    oracle's own state (fields, walkers)."""
    fo = o.fields()
    fluid = _fluid_mask(o.n, o_bc(o))
    rho, u, eps, us = fo["rho"][fluid], fo["u"][:, fluid], fo["eps"][fluid], fo["us"][:, fluid]
    cell, off, img = o.walkers()
    n = np.asarray(o.n)
    X = np.stack([cell % n[0], (cell // n[0]) % n[1], cell // (n[0] * n[1])]).astype(float) + img * n[:, None] + off
    dx = X - o.ref()[:, None]
    se, s1e = eps.sum(), (1.0 - eps).sum()
    return dict(n_walkers=cell.size, n_fluid=int(rho.size),
                sum=np.abs(dx).sum(1), sumsq=(dx * dx).sum(1), mass=np.abs(rho).sum(),
                momentum=np.abs(rho * u).sum(1),
                fluid_u=np.abs((1.0 - eps) * u).sum(1) / s1e if s1e > 0 else np.zeros(3),
                particle_v=np.abs(eps * us).sum(1) / se if se > 0 else np.zeros(3),
                solid_volume=np.abs(eps).sum())


def o_bc(o):
    return o.bc


def _fluid_mask(n, bc):
    m = np.ones(n[::-1], bool)
    for a in range(3):
        if bc[a] == "wall":
            idx = [slice(None)] * 3
            idx[2 - a] = 0
            m[tuple(idx)] = False
            idx[2 - a] = n[a] - 1
            m[tuple(idx)] = False
    return m


def compare(o, g, fields=True, f=True, walkers=True, mom=True):
    if fields:
        fo = o.fields()
        ug, rg = g.velocity()
        _same(ug, fo["u"], "velocity")
        _same(rg, fo["rho"], "density")
    if f:
        # wall nodes hold no distributions (unspecified by the ABI)
        fluid = _fluid_mask(o.n, o_bc(o))
        _same(g.distributions()[:, fluid], o.f()[:, fluid], "distributions")
    if walkers:
        co, oo, io = o.walkers()
        cg, og, ig = g.walkers()
        assert cg.size == co.size
        assert np.array_equal(cg, co), "cells differ for %d walkers" % int(np.count_nonzero(cg != co))
        assert np.array_equal(ig, io), "image counts differ"
        _same(og, oo, "offsets")
        assert np.array_equal(g.occupancy(), o.occupancy()), "occupancy differs"
    if mom:
        mo = o.moments()
        mg = g.moments()
        assert mg["n_walkers"] == int(mo["n_walkers"])
        sc = _moment_scales(o)
        for k in ("sum", "sumsq"):
            _sum_close(mg[k], mo[k], sc[k], sc["n_walkers"], "moment " + k)
        for k in ("momentum", "mass", "solid_volume"):
            _sum_close(mg[k], mo[k], sc[k], sc["n_fluid"], "moment " + k)
        for k in ("fluid_u", "particle_v"):
            _sum_close(mg[k], mo[k], sc[k], sc["n_fluid"], "moment " + k, ratio=True)
        assert mg["counters"] == o.counters()


def test_normals_bitwise(orc, B):
    n = 200_000
    for t, purpose, seed in ((0, 0, 0), (7, 0, 12345), (123, 1, 2**40 + 3), (4999, 2, 2)):
        zg = B.device_normals(seed, t, purpose, n)
        zo = orc.normals(t, purpose, seed, n)
        assert np.array_equal(zg, zo), "normals differ at %d of %d" % (int(np.count_nonzero(zg != zo)), zg.size)


def test_initial_state(orc, B):
    cfg = W.config_tiny(n=(5, 6, 4), bc=("periodic", "wall", "periodic"), n_walkers=0,
                        wall_u=([[0, 0, 0], [0.01, 0, 0], [0, 0, 0]], [[0, 0, 0], [-0.02, 0, 0.01], [0, 0, 0]]),
                        u0=(0.01, 0.0, -0.005))
    o, g = _pair(orc, B, cfg)
    compare(o, g, walkers=False)


TINY = [
    dict(n=(6, 5, 7), bc=("periodic",) * 3, motion="static", n_walkers=200),
    dict(n=(9, 4, 11), bc=("periodic", "wall", "periodic"), motion="sinusoid", n_walkers=300),
    dict(n=(7, 6, 5), bc=("wall", "periodic", "wall"), motion="const_vel", n_walkers=250, spread=0.8),
    dict(n=(8, 8, 8), bc=("wall", "wall", "wall"), motion="sinusoid", n_walkers=400, n_particles=2, spread=1.2),
    dict(n=(10, 7, 9), bc=("periodic", "wall", "periodic"), motion="sinusoid", n_walkers=500, n_particles=3,
         wall_u=([[0, 0, 0], [-0.01, 0, 0], [0, 0, 0]], [[0, 0, 0], [0.02, 0, 0.0], [0, 0, 0]]), D=0.05),
    dict(n=(5, 5, 5), bc=("periodic",) * 3, motion="sinusoid", n_walkers=300, n_particles=2, amp=2.5, period=12.0,
         D=0.002, spread=1.0),
    dict(n=(3, 9, 1), bc=("periodic", "wall", "periodic"), motion="static", n_walkers=50, n_particles=0),
]


@pytest.mark.parametrize("streaming", [1, 2])
@pytest.mark.parametrize("case", range(len(TINY)))
def test_tiny_fp64_parity(orc, B, case, streaming):
    """Both lattice layouts (two lattices; one lattice streamed in place, whose
    slots alternate with the step parity) against the oracle, distributions
    included, after odd and even step counts."""
    kw = dict(TINY[case])
    steps = kw.pop("steps", 12)
    cfg = W.config_tiny(steps=steps, seed=100 + case, **kw)
    o, g = _pair(orc, B, cfg)
    g.set("streaming", streaming)
    compare(o, g)
    for chunk in (1, 3, steps - 4):
        o.step(chunk)
        g.step(chunk)
        compare(o, g)


def test_sweeping_particle_types_2_and_4(orc, B):
    """A particle moving at 0.1 cell/step through slow walkers exercises the
    refill (type II) and the reflection (type IV) paths."""
    cfg = W.config_tiny(n=(16, 12, 12), bc=("periodic",) * 3, n_particles=1, n_walkers=3000, motion="const_vel",
                        D=0.0005, spread=0.8, seed=3, F=(0, 0, 0))
    cfg["particles"][0]["vel"] = np.array([0.1, 0.0, 0.02])
    o, g = _pair(orc, B, cfg)
    for _ in range(4):
        o.step(5)
        g.step(5)
        compare(o, g, f=False)
    c = o.counters()
    assert c["type2"] > 0 and c["type4"] > 0


@pytest.mark.parametrize("n,bc", [((9, 6, 10), ("periodic", "wall", "periodic")),
                                  ((3, 7, 4), ("periodic", "periodic", "wall"))])
def test_long_steps_near_particles(orc, B, n, bc):
    """D = 0.5 (sqrt(2D) = 1): many steps are longer than a cell on some axis,
    so the fast path must look up the end point's coarse-mask word as well
    (shorter steps rely on the start word's dilated block); the second lattice
    is narrower than a coarse block on two axes."""
    cfg = W.config_tiny(n=n, bc=bc, n_particles=3, n_walkers=600, D=0.5, spread=1.0, seed=21, steps=8)
    o, g = _pair(orc, B, cfg)
    for chunk in (1, 3, 4):
        o.step(chunk)
        g.step(chunk)
        compare(o, g)


def test_maximum_particle_count(orc, B):
    """64 overlapping metaballs (the limit): every bit of the cull and mask
    words, full-wave ballots in the prologue, the lowest-index rule where
    particles overlap."""
    cfg = W.config_tiny(n=(20, 18, 22), bc=("periodic", "wall", "periodic"), n_particles=64, n_walkers=3000,
                        D=0.05, spread=0.7, seed=31, steps=6, amp=1.0)
    assert len(cfg["particles"]) == 64
    o, g = _pair(orc, B, cfg)
    for chunk in (1, 2, 3):
        o.step(chunk)
        g.step(chunk)
        compare(o, g)
    c = o.counters()
    assert c["type2"] > 0 and c["type4"] > 0


def test_forced_bisection_failure(orc, B):
    cfg = W.config_plain_fp64(scale=0.2)
    cfg["domain"]["D"] = 0.05
    o, g = _pair(orc, B, cfg)
    o.set_max_bisect(1)
    g.set("max_bisect", 1)
    o.step(10)
    g.step(10)
    compare(o, g, f=False)
    assert o.counters()["bisect_fail"] > 0


def test_plain_fp64_32cubed_full_run(orc, B):
    """The 32^3 configuration (static metaball, body force, 1e4 walkers,
    200 steps) element by element at several points of the run."""
    cfg = W.config_plain_fp64()
    o, g = _pair(orc, B, cfg)
    done = 0
    for chunk in (1, 49, 150):
        o.step(chunk)
        g.step(chunk)
        done += chunk
        compare(o, g)
    assert done == cfg["steps"]


def test_channel_128_fp64_prefix(orc, B):
    """Full-size 128^3 channel (walls, 20 oscillating metaballs, 1e6
    walkers) in FP64 mode: first steps compared element by element."""
    cfg = W.config_channel(precision="fp64")
    o, g = _pair(orc, B, cfg)
    for chunk in (1, 2):
        o.step(chunk)
        g.step(chunk)
        compare(o, g, f=False)


def test_channel_128_fp32_headline(orc, B):
    """The benchmarked configuration itself (128^3 FP32 channel, 20
    oscillating metaballs, 1e6 walkers; default launch shape, one lattice
    streamed in place, walkers regrouped before the first step) against the
    FP64 oracle after 4 steps: velocity within the FP32 bound, walker
    positions within 1e-4 cell for 99.9% of walkers, counts exact."""
    cfg = W.config_channel(precision="fp32")
    o, g = _pair(orc, B, cfg)
    for chunk in (1, 3):
        o.step(chunk)
        g.step(chunk)
    ug, _ = g.velocity()
    uo = o.fields()["u"]
    rel = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
    assert rel < 1e-4, rel
    co, oo, io = o.walkers()
    cg, og, ig = g.walkers()
    n = cfg["domain"]["n"]
    L = np.array(n)[:, None]
    X = lambda c, off, im: np.stack([c % n[0], (c // n[0]) % n[1], c // (n[0] * n[1])]) + off + L * im
    d = np.abs(X(cg, og, ig) - X(co, oo, io))
    assert np.quantile(d.max(0), 0.999) < 1e-4, np.quantile(d.max(0), 0.999)
    assert g.moments()["n_walkers"] == cfg["walkers"]["n"]
    assert int(g.occupancy().sum()) == cfg["walkers"]["n"]


# Stated bounds of the storage modes against FP64 (tests/test_gpu_precision.py
# holds the same values for the 500-step comparison): velocity L2 relative,
# 99th percentile of the walker position error (cells); and, element by
# element, the velocity error relative to max |u|: at most 19 populations of
# magnitude |delta f| <= 1e-3 each carry half an ulp of the storage format
# (2^-11 relative for FP16, 2^-8 for BF16), which gives 1.5e-3 and 1.2e-2 of a
# velocity of 5e-3 (the particles' peak speed); the bounds are three times that.
# FP32 storage rounds at 2^-24: 19 x 1e-3 x 2^-24 is 2.3e-7 of that velocity,
# and the float collision adds rounding of the same order; the bound is 1e-5.
LOWP_BOUNDS = {"fp32": dict(vel_l2=5e-5, pos_p99=2e-5, vel_max=1e-5),
               "fp16": dict(vel_l2=3e-3, pos_p99=3e-4, vel_max=5e-3),
               "bf16": dict(vel_l2=1.5e-2, pos_p99=3e-3, vel_max=4e-2)}


@pytest.fixture(scope="module")
def oscillator_oracle_2steps(orc):
    """The FP64 oracle of the 256^3 oscillator (64 oscillating metaballs, 1e7
    walkers in the solute band) after 2 steps: velocity and walker positions."""
    from paper_2308_05007_amd import workloads as W2
    cfg = W2.config_oscillator(precision="fp64")
    o = orc.build_domain(cfg)
    w = cfg["walkers"]
    assert o.seed(w, w["n"]) == w["n"]
    o.step(2)
    out = dict(u=o.fields()["u"], walkers=o.walkers(), n=cfg["domain"]["n"])
    del o
    return out


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_oscillator_256_lowp_full_size(oscillator_oracle_2steps, B, prec):
    """The benchmarked 256^3 oscillator at its full size (the headline FP32
    storage, and 16-bit storage of deviations; default launch shape, two
    lattices) against the FP64 oracle after 2 steps, within the mode's stated
    bounds: velocity L2, velocity element by element, the 99th percentile of
    the walker position error; walker count and occupancy sum exact."""
    ref = oscillator_oracle_2steps
    cfg = W.config_oscillator(precision=prec)
    g = B.build_domain(cfg)
    g.step(1)
    g.step(1)
    ug, _ = g.velocity()
    uo = ref["u"]
    rel = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
    vmax = float(np.max(np.abs(ug - uo)) / np.max(np.abs(uo)))
    co, oo, io = ref["walkers"]
    cg, og, ig = g.walkers()
    n = ref["n"]
    L = np.array(n)[:, None]
    X = lambda c, off, im: np.stack([c % n[0], (c // n[0]) % n[1], c // (n[0] * n[1])]) + off + L * im
    d = np.sqrt(((X(cg, og, ig) - X(co, oo, io)) ** 2).sum(0))
    bd = LOWP_BOUNDS[prec]
    print("oscillator 256^3 %s vs oracle: velocity L2 %.3g, max |du|/max|u| %.3g, position p50 %.3g p99 %.3g max %.3g"
          % (prec, rel, vmax, np.median(d), np.quantile(d, 0.99), d.max()))
    assert rel < bd["vel_l2"], rel
    assert vmax < bd["vel_max"], vmax
    assert np.quantile(d, 0.99) < bd["pos_p99"], np.quantile(d, 0.99)
    assert g.moments()["n_walkers"] == cfg["walkers"]["n"]
    assert int(g.occupancy().sum()) == cfg["walkers"]["n"]
    g.close()


def test_batch_fp64_against_oracle(orc, B):
    """Nine uneven FP64 simulations stepped as one batch (members of the
    48^3-96^3 shape sweep with fewer walkers, ragged and wall-bounded small
    lattices; four of them on two lattices, the rest in place, so the batch
    runs both layout groups; each member with its own block size of 128, 256
    or 512, as a per-size-class launch shape sets them), the steps replayed
    from captured graphs of 7 and 13 steps: every member equals its own
    oracle run bit for bit."""
    cfgs = []
    for i in (0, 3, 5):
        c = W.config_batch_member(i, precision="fp64", steps=20)
        c["walkers"]["n"] = 20_000
        cfgs.append(c)
    for k, (n, bc, npart, nw) in enumerate((((33, 47, 29), ("periodic",) * 3, 2, 3000),
                                           ((50, 40, 44), ("periodic", "wall", "periodic"), 3, 4000),
                                           ((40, 36, 52), ("wall", "periodic", "wall"), 2, 2500),
                                           ((17, 9, 11), ("periodic", "wall", "periodic"), 1, 700),
                                           ((56, 48, 40), ("periodic",) * 3, 0, 1500),
                                           ((48, 56, 48), ("periodic",) * 3, 2, 0))):
        cfgs.append(W.config_tiny(n=n, bc=bc, n_particles=npart, n_walkers=nw, seed=200 + k, spread=1.5, amp=2.0,
                                  period=30.0, D=0.02, precision="fp64"))
    pairs = [_pair(orc, B, c) for c in cfgs]
    for k, (o, g) in enumerate(pairs):
        if k % 2 == 1:
            g.set("streaming", 1)  # two lattices
    bt = B.Batch()
    for _, g in pairs:
        bt.add(g)
    bt.set("use_graph", 1)
    bt.set("member_blocks", 1)
    for k, (_, g) in enumerate(pairs):
        g.set("block", (128, 256, 512)[k % 3])
    for chunk in (7, 13):
        bt.step(chunk)
        bt.sync()
        for o, g in pairs:
            o.step(chunk)
    for k, (o, g) in enumerate(pairs):
        compare(o, g)
    bt.close()
    for _, g in pairs:
        g.close()


@pytest.mark.parametrize("bs", [128, 256, 512])
@pytest.mark.parametrize("flags", [0, 1, 2, 3])
def test_launch_shapes_match_oracle(orc, B, bs, flags):
    """Every block size and role map of the fused step launch (walker blocks
    interleaved with fluid blocks, per XCD or over the whole grid; uneven
    role counts per XCD) gives the oracle's FP64 result; the steps are
    enqueued in uneven groups so that group edges (fluid-only first launch,
    walker-only last launch) fall at different steps."""
    cfg = W.config_tiny(n=(24, 10, 17), bc=("periodic", "wall", "periodic"), n_particles=3, n_walkers=3000,
                        seed=11, spread=1.5)
    o, g = _pair(orc, B, cfg)
    g.set("block", bs)
    g.set("step_flags", flags)
    for chunk in (5, 1, 6):
        o.step(chunk)
        g.step(chunk)
    compare(o, g, f=False)


@pytest.mark.parametrize("every", [1, 3])
def test_walker_regrouping_keeps_oracle_results(orc, B, every):
    """Regrouping the walkers by coarse block (here before every launch, or
    every third) moves them between slots; ids travel with them, so the FP64
    results by id still equal the oracle's."""
    cfg = W.config_tiny(n=(20, 9, 14), bc=("periodic", "wall", "periodic"), n_particles=2, n_walkers=2500,
                        seed=13, spread=1.5)
    o, g = _pair(orc, B, cfg)
    g.set("sort_every", every)
    for chunk in (4, 7):
        o.step(chunk)
        g.step(chunk)
    compare(o, g, f=False)


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_walker_order_never_shows(B, prec):
    """Moments, walkers and counters are identical whether the walkers are
    never regrouped, regrouped every step or every 5 steps, eager or from a
    graph: every read-out goes by walker id."""
    cfg = W.config_tiny(n=(16, 12, 10), bc=("periodic", "wall", "periodic"), n_particles=3, n_walkers=4000,
                        seed=17, spread=1.5, precision=prec)
    res = []
    for every, graph in ((0, 0), (1, 0), (5, 1)):
        d = B.build_domain(cfg)
        d.set("sort_every", every)
        d.set("use_graph", graph)
        d.step(23)
        m = d.moments()
        res.append((m["sum"].tolist(), m["sumsq"].tolist(), m["counters"], d.walkers(), d.occupancy()))
        d.close()
    for r in res[1:]:
        assert r[0] == res[0][0] and r[1] == res[0][1] and r[2] == res[0][2]
        assert all(np.array_equal(x, y) for x, y in zip(r[3], res[0][3]))
        assert np.array_equal(r[4], res[0][4])


def test_streaming_layout_is_fixed_after_the_first_step(B):
    from paper_2308_05007_amd.binding import RwmiError
    d = B.build_domain(W.config_tiny())
    d.step(1)
    with pytest.raises(RwmiError):
        d.set("streaming", 1)
    d.close()


def test_graph_replay_equals_eager(B):
    cfg = W.config_tiny(n=(9, 4, 11), bc=("periodic", "wall", "periodic"), n_walkers=500, n_particles=2, seed=5)
    a = B.build_domain(cfg)
    b = B.build_domain(cfg)
    b.set("use_graph", 1)
    # one replay; a replay of 64 then 36 eager steps; a new capture of 3
    for n in (37, 100, 3):
        a.step(n)
        b.step(n)
        ua, ra = a.velocity()
        ub, rb = b.velocity()
        assert np.array_equal(ua, ub) and np.array_equal(ra, rb)
        assert all(np.array_equal(x, y) for x, y in zip(a.walkers(), b.walkers()))
        ma, mb = a.moments(), b.moments()
        assert ma["mass"] == mb["mass"] and np.array_equal(ma["momentum"], mb["momentum"])
        assert ma["counters"] == mb["counters"]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_batch_equals_alone(B, prec):
    cfgs = [W.config_tiny(n=n, bc=bc, n_walkers=nw, n_particles=npart, seed=s, precision=prec)
            for n, bc, nw, npart, s in (((9, 4, 11), ("periodic", "wall", "periodic"), 300, 2, 1),
                                         ((6, 6, 6), ("periodic",) * 3, 0, 1, 2),
                                         ((12, 5, 7), ("periodic",) * 3, 700, 3, 3))]
    alone = [B.build_domain(c) for c in cfgs]
    mixed = [B.build_domain(c) for c in cfgs]
    for d in alone:
        d.step(15)
    bt = B.Batch()
    for d in mixed:
        bt.add(d)
    bt.set("use_graph", 1)
    bt.step(15)
    bt.sync()
    for a, m in zip(alone, mixed):
        ua, ra = a.velocity()
        um, rm = m.velocity()
        assert np.array_equal(ua, um) and np.array_equal(ra, rm)
        for x, y in zip(a.walkers(), m.walkers()):
            assert np.array_equal(x, y)
        assert a.moments()["counters"] == m.moments()["counters"]
    bt.close()



def test_large_batch_streams_between_two_lattices_and_equals_alone(B):
    """Members whose distributions together exceed the in-place limit (six
    96^3 FP32 sweep members, 403 MB) are switched to two lattices before
    their first step; each still equals the same simulation run alone in
    place, bit for bit (velocity, density, walkers, counters)."""
    from paper_2308_05007_amd import autotune
    members = [i for i in range(64) if max(W.config_batch_member(i, steps=8)["domain"]["n"]) == 96][:6]
    cfgs = [W.config_batch_member(i, steps=8) for i in members]
    assert autotune.batch_streaming(cfgs) == 1
    print("members", members, flush=True)
    bt, doms = autotune.build_batch(cfgs, use_graph=True)
    bt.step(8)
    bt.sync()
    for i in (0, len(cfgs) - 1):
        a = B.build_domain(cfgs[i])  # alone: 67 MB of distributions, in place
        a.step(8)
        a.sync()
        ua, ra = a.velocity()
        um, rm = doms[i].velocity()
        assert np.array_equal(ua, um) and np.array_equal(ra, rm), i
        for x, y in zip(a.walkers(), doms[i].walkers()):
            assert np.array_equal(x, y), i
        assert a.moments()["counters"] == doms[i].moments()["counters"]
        a.close()
    bt.close()
    for d in doms:
        d.close()


def test_destroy_domain_in_batch(B):
    """Destroying a member takes it out of its batch; the others step on
    exactly as they would alone (graph replay before and after)."""
    cfgs = [W.config_tiny(n=n, bc=bc, n_walkers=nw, n_particles=npart, seed=s)
            for n, bc, nw, npart, s in (((9, 4, 11), ("periodic", "wall", "periodic"), 300, 2, 4),
                                         ((6, 6, 6), ("periodic",) * 3, 200, 1, 5),
                                         ((12, 5, 7), ("periodic",) * 3, 700, 3, 6))]
    alone = [B.build_domain(c) for c in cfgs]
    mixed = [B.build_domain(c) for c in cfgs]
    for d in alone:
        d.step(12)
    bt = B.Batch()
    for d in mixed:
        bt.add(d)
    bt.set("use_graph", 1)
    bt.step(5)
    mixed[1].close()
    assert len(bt.members) == 2
    bt.step(7)
    bt.sync()
    for a, m in ((alone[0], mixed[0]), (alone[2], mixed[2])):
        ua, ra = a.velocity()
        um, rm = m.velocity()
        assert np.array_equal(ua, um) and np.array_equal(ra, rm)
        for x, y in zip(a.walkers(), m.walkers()):
            assert np.array_equal(x, y)
        assert a.moments()["counters"] == m.moments()["counters"]
    bt.close()
    mixed[0].close()
    mixed[2].close()

def test_fp32_mode_against_oracle(orc, B):
    """FP32 storage of deviations, float collision and float walker offsets
    with the same normals: stated bounds after 50 steps of the 32^3 case."""
    cfg = W.config_plain_fp64()
    cfg["domain"]["precision"] = "fp32"
    o, g = _pair(orc, B, cfg)
    o.step(50)
    g.step(50)
    ug, _ = g.velocity()
    uo = o.fields()["u"]
    rel = np.linalg.norm(ug - uo) / np.linalg.norm(uo)
    assert rel < 1e-4, rel
    co, oo, _ = o.walkers()
    cg, og, _ = g.walkers()
    n = cfg["domain"]["n"]
    X = lambda c, off: np.stack([c % n[0], (c // n[0]) % n[1], c // (n[0] * n[1])]) + off
    d = np.abs(X(cg, og) - X(co, oo))
    d = np.minimum(d, n[0] - d)
    assert np.quantile(d.max(0), 0.999) < 1e-4
    assert g.moments()["n_walkers"] == cfg["walkers"]["n"]
