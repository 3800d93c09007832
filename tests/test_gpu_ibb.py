"""Parity of the interpolated bounce-back coupling (Sec. 2.4.3, Eq. 23-27) on
the GPU with the FP64 oracle, through the C ABI.

FP64 runs the oracle's operation sequence (the link fraction q by the same
regula falsi steps, Eq. 24-25 in the same order), so the node status, velocities,
densities, walkers, counters and the distributions of every node that is
fluid after the last update must match bit for bit (the populations of a
solid node are not defined); with coupled particles so must the particle
states, the force now being the links' Galilean-invariant exchange.  Cases:
moving particles that cover and uncover nodes (refill, Eq. 27) with walls,
moving walls and a body force on ragged lattices; a static particle in a
driven flow; coupled particles that collide; 130 steps through a captured
graph; the coupled oscillator of Sec. 4 at full size.  FP32 within bounds
derived from the float rounding of the stored populations."""
import math

import numpy as np
import pytest

from paper_2308_05007_amd import workloads as W
from test_gpu_parity import _fluid_mask, _pair, _same, compare

pytestmark = pytest.mark.gpu

KEYS = ("c", "v", "q", "L", "w", "Fh", "Th", "mass", "I")


@pytest.fixture(scope="module")
def B():
    from paper_2308_05007_amd import binding
    binding.lib()
    return binding


def _ibb(cfg):
    cfg["domain"]["coupling"] = "ibb"
    return cfg


def _compare_ibb(o, g, walkers=True):
    compare(o, g, f=False, walkers=walkers)
    sm = o.smap()
    fluid = _fluid_mask(o.n, o.bc) & (sm == 0)
    _same(g.distributions()[:, fluid], o.f()[:, fluid], "distributions of fluid nodes")
    return sm


def _states(o, g, cfg):
    for p, part in enumerate(cfg["particles"]):
        if part.get("motion") != "coupled":
            continue
        so, sg = o.dem_state(p), g.particle_state(p)
        for k in KEYS:
            _same(sg[k], so[k], "particle %d %s" % (p, k))


CASES = {
    "moving_walls_force": dict(n=(18, 15, 20), bc=("periodic", "wall", "periodic"), n_particles=3, spread=1.8,
                               amp=1.5, period=60.0, steps=24, wall_u=((0, 0, 0, 0.02, 0, 0, 0, 0, 0),
                                                                       (0, 0, 0, -0.01, 0, 0.005, 0, 0, 0))),
    "periodic_sinusoid": dict(n=(20, 18, 22), bc=("periodic",) * 3, n_particles=4, spread=2.2, amp=1.5,
                              period=50.0, steps=30, seed=11),
    "const_vel_walls": dict(n=(17, 19, 16), bc=("wall", "periodic", "wall"), n_particles=2, spread=1.5,
                            motion="const_vel", steps=20, seed=4, D=0.1),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_ibb_prescribed_fp64_bitwise(orc, B, case):
    cfg = _ibb(W.config_tiny(n_walkers=800, **CASES[case]))
    o, g = _pair(orc, B, cfg)
    print("ibb case", case, flush=True)
    steps = cfg["steps"]
    o.step(steps // 2)
    g.step(steps // 2)
    g.sync()
    sm1 = _compare_ibb(o, g)
    o.step(steps - steps // 2)
    g.step(steps - steps // 2)
    g.sync()
    sm2 = _compare_ibb(o, g)
    assert (sm2 > 0).any()
    if case != "const_vel_walls":
        assert np.count_nonzero((sm1 > 0) != (sm2 > 0)) > 0  # nodes were covered and uncovered


def test_ibb_static_particle_in_driven_flow(orc, B):
    cfg = _ibb(W.config_plain_fp64())
    cfg["walkers"]["n"] = 5000
    o, g = _pair(orc, B, cfg)
    o.step(40)
    g.step(40)
    g.sync()
    _compare_ibb(o, g)


def test_ibb_coupled_particles_fp64_bitwise(orc, B):
    cfg = _ibb(W.config_coupled_small(seed=3))
    o, g = _pair(orc, B, cfg)
    o.step(20)
    g.step(20)
    g.sync()
    _states(o, g, cfg)
    o.step(20)
    g.step(20)
    g.sync()
    _states(o, g, cfg)
    _compare_ibb(o, g)
    assert np.abs(o.dem_state(0)["Fh"]).max() > 0


def test_ibb_graph_replay(orc, B):
    cfg = _ibb(W.config_tiny(n=(16, 14, 18), bc=("periodic",) * 3, n_particles=3, spread=1.8, amp=1.5,
                             period=60.0, n_walkers=500, seed=21))
    o, g = _pair(orc, B, cfg)
    g.set("use_graph", 1)
    o.step(130)
    g.step(130)
    g.sync()
    _compare_ibb(o, g)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ibb_coupled_oscillator_full_size(orc, B, precision):
    """The coupled oscillator of Sec. 4 (120 x 120 x 180, 50 particles) with
    bounce-back coupling for 3 steps: FP64 bit for bit; FP32 velocities
    within 1e-6 + 1e-4 |u| of the oracle (a float population carries 2^-24
    of its value, about 3e-9 for w rho0 = 1/18, and the velocity sums 19 of
    them over rho) but at nodes whose solid/fluid status float decides
    differently (at most 1e-5 of them, within 5% of the flow's scale), the
    particle forces within 2e-3 of their scale."""
    cfg = _ibb(W.config_coupled_oscillator(R=5.0, n_walkers=100_000, steps=3, precision=precision))
    o, g = _pair(orc, B, cfg)
    o.step(3)
    g.step(3)
    g.sync()
    if precision == "fp64":
        _states(o, g, cfg)
        compare(o, g, f=False)
    else:
        uo = o.fields()["u"]
        ug, _ = g.velocity()
        # float takes the solid/fluid decision of a node and the link fraction
        # in float: where a node centre sits within float rounding of a
        # surface, its status (and its neighbours' links) can differ from
        # FP64's; such nodes are rare and their velocities stay within a few
        # percent of the flow's scale
        bad = np.abs(ug - uo) > 1e-6 + 1e-4 * np.abs(uo)
        assert np.count_nonzero(bad) <= 1e-5 * bad.size, np.count_nonzero(bad)
        assert np.abs(ug - uo).max() <= 0.05 * np.abs(uo).max()
        for p in range(len(cfg["particles"])):
            so, sg = o.dem_state(p), g.particle_state(p)
            assert np.abs(sg["Fh"] - so["Fh"]).max() <= 2e-3 * np.abs(so["Fh"]).max() + 1e-9, p


@pytest.mark.parametrize("precision,rel", [("fp16", 0.01), ("bf16", 0.05)])
def test_ibb_half_storage_within_bounds(orc, B, precision, rel):
    """FP16 and BF16 storage of the deviations f - w rho0 with bounce-back
    (moving particles that cover and uncover nodes, 30 steps): a stored
    deviation of about 3 w rho0 |u| carries a relative rounding of 2^-11
    (FP16) or 2^-8 (BF16), some 1e-5 and 1e-4 of the flow's velocity scale
    per step, so after 30 steps the velocities stay within 1% (FP16) and
    5% (BF16) of the largest velocity at 99.9% of the nodes (the rest being
    nodes whose solid/fluid status float decides differently) and within 10%
    everywhere; the densities within the same fractions of the largest
    density deviation plus 1e-4."""
    cfg = _ibb(W.config_tiny(n_walkers=200, precision=precision, **CASES["periodic_sinusoid"]))
    o, g = _pair(orc, B, cfg)
    print("ibb half storage", precision, flush=True)
    o.step(cfg["steps"])
    g.step(cfg["steps"])
    g.sync()
    uo = o.fields()["u"]
    ug, rg = g.velocity()
    scale = np.abs(uo).max()
    assert scale > 1e-3
    err = np.abs(ug - uo).max(axis=0)
    assert np.count_nonzero(err > rel * scale) <= max(1, 1e-3 * err.size), np.sort(err.ravel())[-5:] / scale
    assert err.max() <= 0.1 * scale
    ro = o.fields()["rho"]
    dscale = np.abs(ro - 1.0).max()
    rerr = np.abs(rg - ro)
    assert np.count_nonzero(rerr > rel * dscale + 1e-4) <= max(1, 1e-3 * rerr.size)


def test_ibb_control_points_beyond_the_lds_table(orc, B):
    """40 particles of 30 control points (1200 in all, more than the link
    pass holds in LDS, so it reads them from global memory): FP64 bit for
    bit, with nodes covered and uncovered."""
    cfg = _ibb(W.config_tiny(n=(24, 20, 22), bc=("periodic",) * 3, n_particles=40, n_walkers=300, amp=1.5,
                             period=40.0, seed=31, steps=16))
    rng = np.random.default_rng(77)
    for p in cfg["particles"]:
        b, k = W.metaball_shape(rng, 30, 1.0, (0.03, 0.06))
        p["b"], p["k"] = b, k
    assert sum(len(p["k"]) for p in cfg["particles"]) > 1024
    o, g = _pair(orc, B, cfg)
    print("ibb 1200 control points", flush=True)
    o.step(8)
    g.step(8)
    g.sync()
    sm1 = _compare_ibb(o, g)
    o.step(8)
    g.step(8)
    g.sync()
    sm2 = _compare_ibb(o, g)
    assert (sm2 > 0).any() and np.count_nonzero((sm1 > 0) != (sm2 > 0)) > 0


def test_ibb_without_particles_is_plain_bgk(orc, B):
    """No particle at all: nothing is ever solid, the link pass finds no
    link, and the bounce-back domain advances exactly as the oracle's (and
    as plain BGK with walls and a body force)."""
    cfg = _ibb(W.config_tiny(n=(13, 11, 9), bc=("periodic", "wall", "periodic"), n_particles=0, n_walkers=100,
                             steps=12, wall_u=((0, 0, 0, 0.01, 0, 0, 0, 0, 0), (0, 0, 0, 0, 0, 0, 0, 0, 0))))
    o, g = _pair(orc, B, cfg)
    o.step(12)
    g.step(12)
    g.sync()
    sm = _compare_ibb(o, g)
    assert not (sm > 0).any()


def _array_flow(B, coupling, R, L=48, f=1e-7, tau=0.8, steps=30000):
    """Mean velocity of body-force-driven flow through a simple cubic array
    of spheres (one static one-point metaball, M = R^2 / r^2, in a periodic
    L^3 box), extrapolated to the steady state by Aitken's delta-squared over
    the last three samples (the mean flow approaches it as one exponential,
    time constant about 6000 steps here)."""
    dom = W._domain((L, L, L), ("periodic",) * 3, tau, (f, 0, 0), 0.0, seed=1, precision="fp64")
    if coupling == "ibb":
        dom["coupling"] = "ibb"
    cfg = dict(name="array", domain=dom, walkers=dict(kind="uniform", n=0), steps=steps,
               particles=[dict(b=np.zeros((1, 3)), k=np.array([R * R]), centre=np.array([L / 2] * 3),
                               motion="static")])
    g = B.build_domain(cfg, device=0)
    g.set("use_graph", 1)
    us = []
    for _ in range(steps // 2000):
        g.step(2000)
        g.sync()
        us.append(float(g.velocity()[0][0].mean()))
    g.close()
    a, b, c = us[-3:]
    return (a * c - b * b) / (a + c - 2 * b)


@pytest.mark.parametrize("R", [4.0, 6.0])
def test_sphere_array_drag_against_sangani_acrivos(B, R):
    """The comparison the bounce-back coupling was built for (Sec. 2.4.3,
    the paper's own coupling against partially saturated cells): Stokes flow
    (Re < 0.1) through a simple cubic array of spheres of volume fraction phi,
    whose drag F = 6 pi mu R U K(phi) has the dilute expansion of Sangani and
    Acrivos (1982), 1/K = 1 - 1.7601 phi^(1/3) + phi - 1.5593 phi^2 +
    3.9799 phi^(8/3) - 3.0734 phi^(10/3); the body force on the fluid
    f L^3 (1 - phi) balances it.  Bounce-back gives the mean velocity U
    within 1.5% of the closed form (0.25% and 0.65% measured at R = 4 and 6),
    partially saturated cells within 6% (4.0% and 2.9% too fast), and
    bounce-back is the closer of the two."""
    L, f, tau = 48, 1e-7, 0.8
    mu = (tau - 0.5) / 3.0
    phi = 4.0 / 3.0 * math.pi * R ** 3 / L ** 3
    K = 1.0 / (1 - 1.7601 * phi ** (1 / 3) + phi - 1.5593 * phi ** 2 + 3.9799 * phi ** (8 / 3)
               - 3.0734 * phi ** (10 / 3))
    U = f * L ** 3 * (1 - phi) / (6 * math.pi * mu * R * K)
    print("sphere array R", R, flush=True)
    ui = _array_flow(B, "ibb", R)
    up = _array_flow(B, "psm", R)
    assert abs(ui / U - 1) < 0.015, (ui / U, up / U)
    assert abs(up / U - 1) < 0.06, (ui / U, up / U)
    assert abs(ui / U - 1) < abs(up / U - 1)
    assert U * 2 * R / mu < 0.1  # Reynolds number (rho = 1)


@pytest.mark.parametrize("kind", ["ibb", "coupled"])
def test_batches_refuse_coupled_domains(B, kind):
    """A domain with the bounce-back coupling or with two-way coupled
    particles steps alone: adding it to a batch is EINVAL, and the batch
    still steps its other members."""
    cfg = _ibb(W.config_tiny()) if kind == "ibb" else W.config_coupled_small(n_walkers=100, steps=2)
    d = B.build_domain(cfg, device=0)
    plain = B.build_domain(W.config_tiny(precision="fp32"), device=0)
    b = B.Batch()
    with pytest.raises(B.RwmiError) as e:
        b.add(d)
    assert e.value.status == B.RWMI_EINVAL
    b.add(plain)
    b.step(2)
    b.sync()
    b.remove(plain)
    b.close()
    plain.close()
    d.close()
