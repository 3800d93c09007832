"""Parity of the two-way coupled particles (Sec. 2.2, Eq. 4-11) on the GPU
with the FP64 oracle, through the C ABI.

FP64: the particle update runs the oracle's sequence of IEEE operations and
the hydrodynamic force is summed in 2^-48 fixed point on both sides, so the
particle states (centre, velocity, quaternion, angular momentum and
velocity, force, torque) must match bit for bit, and with them the
distributions, velocities, walkers and counters (the same checks as the
prescribed-motion parity).  The cases collide two particles (the contact
changes their velocities by more than 0.01 within the run), put a third on
a wall under gravity, mix coupled and prescribed particles, and run through
a captured graph.  FP32: the fluid's force in float, particle states within
bounds derived from the float rounding of the force.  Full size: the
oscillator of Sec. 4 with 50 coupled particles on 120 x 120 x 180 nodes."""
import numpy as np
import pytest

from paper_2308_05007_amd import workloads as W
from test_gpu_parity import _pair, _same, compare

pytestmark = pytest.mark.gpu

KEYS = ("c", "v", "q", "L", "w", "Fh", "Th", "mass", "I")


@pytest.fixture(scope="module")
def B():
    from paper_2308_05007_amd import binding
    binding.lib()
    return binding


def _coupled(cfg):
    return [i for i, p in enumerate(cfg["particles"]) if p.get("motion") == "coupled"]


def _same_states(o, g, cfg, what=""):
    for p in _coupled(cfg):
        so, sg = o.dem_state(p), g.particle_state(p)
        for k in KEYS:
            _same(sg[k], so[k], "%s particle %d %s" % (what, p, k))


def _run(orc, B, cfg, steps, chunks=1):
    o, g = _pair(orc, B, cfg)
    print("coupled case", cfg["name"], cfg["domain"]["n"], cfg["domain"]["precision"], "steps", steps, flush=True)
    _same_states(o, g, cfg, "initial")
    per = steps // chunks
    for _ in range(chunks):
        o.step(per)
        g.step(per)
        g.sync()
    return o, g


@pytest.mark.parametrize("case", ["periodic", "wall_gravity", "mixed"])
def test_coupled_fp64_bitwise(orc, B, case):
    kw = {"periodic": dict(), "wall_gravity": dict(n=(26, 22, 22), bc=("periodic", "periodic", "wall"),
                                                   g=(0, 0, -5e-4), speed=0.05),
          "mixed": dict(with_prescribed=True, seed=5)}[case]
    cfg = W.config_coupled_small(**kw)
    o, g = _run(orc, B, cfg, cfg["steps"], chunks=2)
    _same_states(o, g, cfg)
    compare(o, g)
    v0 = cfg["particles"][0]["vel"]
    assert abs(o.dem_state(0)["v"][0] - v0[0]) > 0.01  # the pair met and the fluid slowed it
    assert g.moments()["contact_misses"] == 0


def test_free_and_candidate_steps_alternate(orc, B):
    """A pair in a periodic box that starts with no contact candidate (the
    particle update runs its substeps without barriers), comes within the
    candidate margin, collides (the synchronised substeps with contacts) and
    separates again: FP64 states bit for bit with the oracle after every 10
    steps through all three phases."""
    cfg = W.config_coupled_small(gap=3.0, speed=0.08, steps=140, n_particles=2)
    cfg["dem"]["rho_p"] = 20.0  # heavy enough to reach the other through the fluid
    o, g = _pair(orc, B, cfg)
    r = sum(W.bounding_radius(p["b"], p["k"]) for p in cfg["particles"])
    n = np.asarray(cfg["domain"]["n"], float)
    gaps = []
    for k in range(14):
        dc = o.dem_state(1)["c"] - o.dem_state(0)["c"]
        dc -= n * np.floor(dc / n + 0.5)
        gaps.append(float(np.linalg.norm(dc)) - r)
        print("chunk", k, "bounding-sphere gap %.3f" % gaps[-1], flush=True)
        o.step(10)
        g.step(10)
        g.sync()
        _same_states(o, g, cfg, "chunk %d" % k)
    compare(o, g)
    # far (no candidate: the candidate margin is 1), in contact, far again
    assert gaps[0] > 2.0 and min(gaps) < -1.0 and gaps[-1] > 2.0, gaps


def test_coupled_graph_equals_eager(orc, B):
    """130 steps through a captured graph of 128 steps and two eager ones:
    the same bits as the oracle."""
    cfg = W.config_coupled_small(seed=11, n=(22, 20, 26), n_walkers=1500, steps=130)
    o, g = _pair(orc, B, cfg)
    g.set("use_graph", 1)
    o.step(130)
    g.step(130)
    g.sync()
    _same_states(o, g, cfg)
    compare(o, g)


def test_set_particle_motion(orc, B):
    """A spin given through the ABI: the same w = R I^-1 R^T L as the oracle
    and the same trajectory."""
    cfg = W.config_coupled_small(seed=7, n_walkers=500, steps=12)
    o, g = _pair(orc, B, cfg)
    o.step(4)
    g.step(4)
    L = np.array([30.0, -12.0, 55.0])
    o.dem_set_motion(1, (0.01, 0.0, -0.02), L)
    g.set_particle_motion(1, (0.01, 0.0, -0.02), L)
    _same_states(o, g, cfg, "after set")
    o.step(8)
    g.step(8)
    g.sync()
    _same_states(o, g, cfg)
    compare(o, g)


def test_coupled_fp32_within_float_bounds(orc, B):
    """FP32 lattice, FP64 particle update: the force is summed from float
    node shares, each within a few float ulps of the FP64 one, so after a
    short run without contacts the states stay within bounds far above the
    accumulated rounding yet far below the motion itself."""
    cfg = W.config_coupled_small(seed=3, gap=2.0, precision="fp32", n_walkers=1000, steps=20)
    o, g = _pair(orc, B, cfg)
    o.step(20)
    g.step(20)
    g.sync()
    for p in _coupled(cfg):
        so, sg = o.dem_state(p), g.particle_state(p)
        dv = np.abs(sg["v"] - so["v"]).max()
        assert dv < 1e-5 * max(1.0, 100 * np.abs(so["v"]).max()), (p, dv)
        assert np.abs(sg["c"] - so["c"]).max() < 1e-4
        assert np.abs(sg["Fh"] - so["Fh"]).max() <= 2e-3 * np.abs(so["Fh"]).max() + 1e-9
        assert np.abs(sg["q"] - so["q"]).max() < 1e-6


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_oscillator_full_size(orc, B, precision):
    """The coupled oscillator of Sec. 4 at full size (R = 5: 120 x 120 x 180
    nodes, 50 particles, 200 000 walkers) for 3 steps: FP64 bit for bit,
    FP32 within the float bounds of the force."""
    cfg = W.config_coupled_oscillator(R=5.0, n_walkers=200_000, steps=3, precision=precision)
    o, g = _run(orc, B, cfg, 3)
    if precision == "fp64":
        _same_states(o, g, cfg)
        compare(o, g, f=False)
    else:
        for p in _coupled(cfg):
            so, sg = o.dem_state(p), g.particle_state(p)
            assert np.abs(sg["Fh"] - so["Fh"]).max() <= 2e-3 * np.abs(so["Fh"]).max() + 1e-9, p
            assert np.abs(sg["v"] - so["v"]).max() <= 1e-3 * np.abs(so["v"]).max() + 1e-12, p
            assert np.abs(sg["c"] - so["c"]).max() < 1e-9 + 1e-3 * np.abs(so["v"]).max() * 3


@pytest.mark.parametrize("coupling", ["psm", "ibb"])
def test_sixty_four_coupled_particles(orc, B, coupling):
    """The largest particle count a domain takes, all two-way coupled (the
    particle update's one wave of 64 lanes full), with either coupling: the
    states bit for bit after 4 steps."""
    cfg = W.config_coupled_oscillator(R=2.0, n_particles=64, n_walkers=2000, steps=4, precision="fp64", seed=5)
    assert len(cfg["particles"]) == 64
    if coupling == "ibb":
        cfg["domain"]["coupling"] = "ibb"
    o, g = _run(orc, B, cfg, 4, chunks=2)
    _same_states(o, g, cfg)
    compare(o, g, f=False)


@pytest.mark.parametrize("precision,eps", [("fp16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
@pytest.mark.parametrize("gap", [2.0, None])
def test_coupled_half_storage_within_bounds(orc, B, precision, eps, gap):
    """Coupled particles over a lattice stored in FP16 or BF16 (particle
    update in FP64), 20 steps, with and without the collision: each stored
    deviation carries a relative rounding of eps = 2^-11 (FP16) or 2^-8
    (BF16), and so do the exchange terms the force sums, so the force stays
    within 4 eps of its scale, the velocities within 2 eps of theirs, the
    positions within 1e-3 cells and the fluid velocity within 4 eps of its
    largest value (measured: at most a fifth of these)."""
    kw = dict(gap=gap) if gap is not None else {}
    cfg = W.config_coupled_small(seed=3, precision=precision, n_walkers=1000, steps=20, **kw)
    o, g = _pair(orc, B, cfg)
    print("coupled", precision, "gap", gap, flush=True)
    o.step(20)
    g.step(20)
    g.sync()
    for p in _coupled(cfg):
        so, sg = o.dem_state(p), g.particle_state(p)
        assert np.abs(sg["Fh"] - so["Fh"]).max() <= 4 * eps * np.abs(so["Fh"]).max() + 1e-12, p
        assert np.abs(sg["v"] - so["v"]).max() <= 2 * eps * np.abs(so["v"]).max() + 1e-12, p
        assert np.abs(sg["c"] - so["c"]).max() < 1e-3, p
    uo = o.fields()["u"]
    ug, _ = g.velocity()
    assert np.abs(ug - uo).max() <= 4 * eps * np.abs(uo).max()
