"""Pins of the oracle parts that the walker and fluid tests leave open:
trilinear velocity interpolation (Sec. 2.4.1), the solid-node collision term
of the partially saturated cell method (reading of Sec. 1 with
Noble-Torczynski weighting), the fluid and particle averages that feed Eq.
39-40, multi-period wrapping of long steps, and the return-to-origin rules
for non-finite and doubly out-of-range positions.

Every test here was run against deliberately broken copies of the oracle on
the CPU and failed on each of them: interpolation weights w and 1 - w
swapped, the base node taken on the wrong side for offsets below 1/2, wall
nodes interpolated with the fluid value instead of the wall velocity, u and
u_s exchanged between the two equilibria of the solid term, the bounced
population taken from direction i instead of its opposite, the (1 - eps)
weight of the fluid average replaced by 1, the particle average taken over
the fluid velocity, a single-period wrap of the cell index, and the
out-of-range return removed."""
import math

import numpy as np
import pytest


# --------------------------------------------------------------- helpers
def _node_centres(n):
    """Node centre coordinates (i + 1/2) of a lattice [z][y][x] as three arrays."""
    zz, yy, xx = np.meshgrid(*(np.arange(v) + 0.5 for v in n[::-1]), indexing="ij")
    return xx, yy, zz


def _prescribe_velocity(orc, o, n, u):
    """Set every node to f^eq(1, u(x)) so that the fluid step of the next
    step computes exactly u (to rounding) as its velocity field."""
    N = int(np.prod(n))
    f = np.empty((19, N))
    ur = u.reshape(3, -1)
    for k in range(N):
        f[:, k] = orc.feq(1.0, ur[:, k])
    o.set_f(f)


def _unwrapped(cell, off, img, n):
    c = np.stack([cell % n[0], (cell // n[0]) % n[1], cell // (n[0] * n[1])], -1).astype(float)
    return c + img.T * np.asarray(n, float) + off.T


def _set_positions(o, X, n, ref):
    c3 = np.floor(X).astype(np.int64)
    cell = (c3[:, 0] + n[0] * (c3[:, 1] + n[1] * c3[:, 2])).astype(np.int32)
    o.set_walkers(cell, (X - c3).T.ravel(), ref)


# ---------------------------------------------------- trilinear velocity
def _interp_1d(p, x, m):
    """Closed form of the piecewise-linear interpolant between node centres
    (spacing 1) of the monomial (X - m)^p, p = 0, 1, 2, at x: exact for p <= 1;
    for p = 2 the chord between the two enclosing centres exceeds the
    parabola by w (1 - w), w the distance of x past the lower centre."""
    w = (x - 0.5) - np.floor(x - 0.5)
    if p == 0:
        return np.ones_like(x)
    if p == 1:
        return x - m
    return (x - m) ** 2 + w * (1.0 - w)


def test_trilinear_interpolation_of_a_quadratic_field(orc):
    """With D = 0 a walker moves by exactly the interpolated velocity (Eq. 2).
    Prescribe on the node centres a field that is a sum of products of
    per-axis monomials of degree <= 2.  Interpolation along x, y and z in turn
    between the eight surrounding centres is the tensor product of the 1-D
    piecewise-linear interpolants, so each walker's displacement has a closed
    form.  The quadratic terms fix which two centres enclose the walker on
    each axis, the linear and cross terms fix the weights of each axis."""
    n = (11, 9, 10)
    m = np.array([5.3, 4.1, 4.9])
    rng = np.random.default_rng(21)
    A = rng.uniform(-1.0, 1.0, (3, 3, 3, 3))  # [component][px][py][pz]
    xx, yy, zz = _node_centres(n)
    C = (xx, yy, zz)
    raw = np.zeros((3,) + xx.shape)
    for c in range(3):
        for p in np.ndindex(3, 3, 3):
            raw[c] += A[(c,) + p] * np.prod([(C[a] - m[a]) ** p[a] for a in range(3)], axis=0)
    scale = 0.05 / np.abs(raw).max()
    u = raw * scale
    o = orc.Oracle(dict(n=n, bc=("periodic",) * 3, tau=0.8, F=(0, 0, 0), D=0.0, seed=3))
    _prescribe_velocity(orc, o, n, u)
    # interior walkers: both enclosing centres of every axis lie inside the box
    N = 3000
    X0 = np.stack([rng.uniform(1.5, n[a] - 1.5, N) for a in range(3)], -1)
    # include offsets exactly at 0, 1/2 and just below 1/2 on every axis
    X0[:6] = np.floor(X0[:6]) + np.array([[0.0], [0.5], [0.5 - 2 ** -40], [0.25], [0.75], [0.999]])
    X0[:6] = np.clip(X0[:6], 1.5, np.array(n) - 1.5 - 1e-9)
    _set_positions(o, X0, n, m)
    o.step(1)
    assert np.max(np.abs(o.fields()["u"] - u)) < 1e-16, np.max(np.abs(o.fields()["u"] - u))
    X1 = _unwrapped(*o.walkers(), n)
    expect = np.zeros((N, 3))
    for c in range(3):
        for p in np.ndindex(3, 3, 3):
            expect[:, c] += A[(c,) + p] * np.prod([_interp_1d(p[a], X0[:, a], m[a]) for a in range(3)], axis=0)
    expect *= scale
    err = np.abs((X1 - X0) - expect)
    assert err.max() < 1e-14, err.max()


def test_interpolation_in_couette_flow_with_wall_nodes(orc):
    """Couette steady state (moving walls, Eq. 23 term): u_x is linear between
    the wall velocities at the halfway planes y = 1 and y = ny - 1 (pinned in
    test_oracle_lbm).  Walkers with D = 0 move by the interpolated u_x: the
    linear profile itself where both enclosing centres are fluid nodes, and
    the chord from the wall node's centre (which carries the wall velocity)
    to the first fluid centre in the half cell next to each wall."""
    ny, U = 12, 0.01
    wl, wh = np.zeros(9), np.zeros(9)
    wl[3], wh[3] = -U, 2 * U
    n = (3, ny, 2)
    o = orc.Oracle(dict(n=n, bc=("periodic", "wall", "periodic"), tau=0.9, F=(0, 0, 0), D=0.0, seed=0,
                        wall_lo=wl, wall_hi=wh))
    o.step(40000)

    def prof(y):
        return -U + 3 * U * (y - 1) / (ny - 2)

    assert np.max(np.abs(o.fields()["u"][0, 0, 1:-1, 0] - prof(np.arange(1, ny - 1) + 0.5))) < 1e-12
    rng = np.random.default_rng(5)
    N = 2000
    y = np.concatenate([rng.uniform(1.0, 1.5, 200), rng.uniform(ny - 1.5, ny - 1.0, 200),
                        rng.uniform(1.5, ny - 1.5, N - 400)])
    X0 = np.stack([rng.uniform(0, n[0], N), y, rng.uniform(0, n[2], N)], -1)
    _set_positions(o, X0, n, (1.5, ny / 2, 1.0))
    o.step(1)
    X1 = _unwrapped(*o.walkers(), n)
    ex = prof(y)
    lo, hi = y < 1.5, y >= ny - 1.5
    ex[lo] = -U + (y[lo] - 0.5) * (prof(1.5) + U)
    ex[hi] = prof(ny - 1.5) + (y[hi] - (ny - 1.5)) * (2 * U - prof(ny - 1.5))
    assert np.max(np.abs((X1[:, 0] - X0[:, 0]) - ex)) < 1e-12
    assert np.max(np.abs(X1[:, 1:] - X0[:, 1:])) < 1e-12


# ------------------------------------------------------ PSM solid term
def _B(eps, tau):
    """Noble-Torczynski weighting of the solid term."""
    return eps * (tau - 0.5) / ((1.0 - eps) + (tau - 0.5))


def _nonequilibrium_part(orc, rng, amp=2e-3):
    """A perturbation g with no mass and no momentum (so the velocity the
    node computes is unchanged), built by projecting random values on the
    lattice moments."""
    e, w = orc.lattice()
    g = amp * rng.standard_normal(19)
    M = np.vstack([np.ones(19), e.T.astype(float)])  # 4 x 19
    return g - M.T @ np.linalg.solve(M @ M.T, M @ g)


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.7])
def test_psm_solid_term_direction_by_direction(orc, tau):
    """f = f^eq(rho, u) + g at a node of solid fraction eps, no force.  The
    relaxation takes (1 - B) of the node towards f^eq(rho, u) with rate
    1/tau and the solid term B replaces the node's own non-equilibrium part
    by its opposite and its equilibrium by f^eq(rho, u_s):
        f*_i = (1 - B) f^eq_i(u) + B f^eq_i(u_s) + (1 - B)(1 - 1/tau) g_i + B g_opp(i).
    At eps = 1 this is f^eq_i(rho, u_s) + g_opp(i) direction by direction."""
    e, _ = orc.lattice()
    rng = np.random.default_rng(int(tau * 100))
    o = orc.Oracle(dict(n=(3, 3, 3), bc=("periodic",) * 3, tau=tau, F=(0, 0, 0), D=0.0, seed=0))
    opp = np.array([0] + [i + 1 if i % 2 else i - 1 for i in range(1, 19)])
    for eps in (0.0, 0.15, 0.5, 0.85, 1.0):
        rho = 1.0 + 0.1 * rng.uniform(-1, 1)
        u = 0.05 * rng.uniform(-1, 1, 3)
        us = 0.05 * rng.uniform(-1, 1, 3)
        g = _nonequilibrium_part(orc, rng)
        f = orc.feq(rho, u) + g
        out, r, uo = o.collide_node(f, eps, us)
        assert abs(r - rho) < 1e-15 and np.allclose(uo, u, rtol=0, atol=1e-16)
        B = _B(eps, tau)
        ref = (1 - B) * orc.feq(rho, u) + B * orc.feq(rho, us) + (1 - B) * (1 - 1 / tau) * g + B * g[opp]
        assert np.max(np.abs(out - ref)) < 2e-16, (eps, np.max(np.abs(out - ref)))
        if eps == 1.0:
            assert np.max(np.abs(out - (orc.feq(rho, us) + g[opp]))) < 2e-16


# ------------------------------------------------------------- moments
def test_poiseuille_fluid_average_and_momentum(orc):
    """At the exact tau the channel profile is u(y) = F/(2 nu)(y - 1)(ny - 1 - y)
    on the H = ny - 2 fluid centres y = j + 1/2.  Its mean over the fluid
    nodes is F/(2 nu) (H^2/6 + 1/12) (sum of (j - 1/2)(H - j + 1/2) over
    j = 1..H is H^3/6 + H/12); with no particles the fluid average of the
    moments is that mean, the mass is the number of fluid nodes and the
    momentum the mass times the mean.  The particle average and the solid
    volume are zero."""
    ny, F = 12, 1e-6
    tau = 0.5 + math.sqrt(3.0) / 4.0
    nx, nz = 2, 3
    o = orc.Oracle(dict(n=(nx, ny, nz), bc=("periodic", "wall", "periodic"), tau=tau, F=(F, 0, 0), D=0.0, seed=0))
    o.step(30000)
    nu = (tau - 0.5) / 3.0
    H = ny - 2
    mean = F / (2 * nu) * (H * H / 6.0 + 1.0 / 12.0)
    m = o.moments()
    nf = nx * H * nz
    assert abs(m["fluid_u"][0] - mean) < 1e-9 * mean
    assert np.all(np.abs(m["fluid_u"][1:]) < 1e-12 * mean)
    assert abs(m["mass"] - nf) < 1e-11 * nf
    assert abs(m["momentum"][0] - nf * mean) < 1e-9 * nf * mean
    assert np.all(m["particle_v"] == 0.0) and m["solid_volume"] == 0.0


def test_averages_with_spheres_in_a_prescribed_flow(orc):
    """Two one-control-point particles (spheres of radius sqrt(k), where the
    solid fraction is the unit ramp clamp(1/2 + sqrt(k) - r, 0, 1)) moving
    at different constant velocities, in a prescribed non-uniform flow.
    After one step the moments hold the flow the step computed (the
    prescribed one) and the solid fraction at the poses of t = 0, so every
    average has a closed form: the fluid average weights u by 1 - eps, the
    particle average weights each particle's velocity by its own solid
    volume, the solid volume is the sum of the ramps."""
    n = (24, 20, 22)
    xx, yy, zz = _node_centres(n)
    u = np.stack([0.02 * np.sin(2 * np.pi * yy / n[1]) + 0.01 * zz / n[2],
                  0.015 * np.cos(2 * np.pi * xx / n[0]),
                  -0.01 * (xx / n[0]) * (yy / n[1])])
    parts = [(np.array([6.3, 7.1, 8.6]), 9.0, np.array([0.01, -0.02, 0.005])),
             (np.array([16.9, 13.4, 14.2]), 12.25, np.array([-0.03, 0.01, 0.02]))]
    o = orc.Oracle(dict(n=n, bc=("periodic",) * 3, tau=0.8, F=(0, 0, 0), D=0.0, seed=0))
    eps_p = []
    for c, k, v in parts:
        o.add_particle(dict(b=np.zeros((1, 3)), k=np.array([k]), centre=c, motion="const_vel", vel=v))
        d = [(C - c[a]) - n[a] * np.floor((C - c[a]) / n[a] + 0.5) for a, C in enumerate((xx, yy, zz))]
        r = np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
        eps_p.append(np.clip(0.5 + math.sqrt(k) - r, 0.0, 1.0))
    assert np.all(eps_p[0] * eps_p[1] == 0.0)  # the supports do not overlap
    _prescribe_velocity(orc, o, n, u)
    o.step(1)
    eps = eps_p[0] + eps_p[1]
    flds = o.fields()
    assert np.max(np.abs(flds["eps"] - eps)) < 1e-13
    m = o.moments()
    V = [e.sum() for e in eps_p]
    assert abs(m["solid_volume"] - (V[0] + V[1])) < 1e-11
    pv = (V[0] * parts[0][2] + V[1] * parts[1][2]) / (V[0] + V[1])
    assert np.allclose(m["particle_v"], pv, rtol=1e-12, atol=0)
    fu = ((1.0 - eps) * u).reshape(3, -1).sum(1) / (1.0 - eps).sum()
    assert np.allclose(m["fluid_u"], fu, rtol=1e-11, atol=1e-17)
    N = int(np.prod(n))
    assert abs(m["mass"] - N) < 1e-11 * N
    assert np.allclose(m["momentum"], u.reshape(3, -1).sum(1), rtol=1e-11, atol=1e-14)


# ------------------------------------------------ long steps, wrap, returns
def test_steps_longer_than_the_period(orc):
    """A 3x3x3 periodic box with sqrt(2D) = 4 cells per axis step: most steps
    cross several periods.  The unwrapped mean squared displacement is still
    6 D t (chi^2_3 spread, 4 sigma), and every stored cell and offset is in
    range, which needs the image count to absorb any number of periods."""
    N, D, t = 20000, 8.0, 12
    n = (3, 3, 3)
    c = (1.25, 1.5, 1.75)
    o = orc.Oracle(dict(n=n, bc=("periodic",) * 3, tau=0.8, F=(0, 0, 0), D=D, seed=17))
    assert o.seed(dict(kind="explicit", xyz=np.tile(c, (N, 1)), ref=c), N) == N
    o.step(t)
    cell, off, img = o.walkers()
    assert cell.min() >= 0 and cell.max() < 27
    assert off.min() >= 0.0 and off.max() < 1.0
    assert np.abs(img).max() > 10
    m = o.moments()
    msd = m["sumsq"].sum() / N
    sd = 6 * D * t * math.sqrt(2.0 / (3 * N))
    assert abs(msd - 6 * D * t) < 4 * sd, (msd, 6 * D * t, sd)
    X = _unwrapped(cell, off, img, n)
    assert abs(((X - np.asarray(c)) ** 2).sum() / N - msd) < 1e-9 * msd


def test_non_finite_velocity_returns_walkers(orc):
    """A node with no mass has no velocity (0/0).  A walker whose step is not
    finite stays where it was and is counted as returned to its origin."""
    n = (5, 4, 6)
    o = orc.Oracle(dict(n=n, bc=("periodic",) * 3, tau=0.8, F=(0, 0, 0), D=0.01, seed=4))
    o.set_f(np.zeros(19 * int(np.prod(n))))
    rng = np.random.default_rng(8)
    X0 = np.stack([rng.uniform(0, n[a], 300) for a in range(3)], -1)
    _set_positions(o, X0, n, (2, 2, 3))
    o.step(1)
    assert np.all(np.isnan(o.fields()["u"]))
    X1 = _unwrapped(*o.walkers(), n)
    assert np.array_equal(X1, X0)
    assert o.counters()["returned_to_origin"] == 300


def test_wall_reflection_out_of_range_returns(orc):
    """Wall axis y with the fluid range [1, ny - 1) of width 4 and steps of
    sqrt(2D) = 3 per axis, in a fluid at rest: the expected end point is
    computed here from the walker's normals (pinned separately).  Below the
    range a point reflects to 2 - y, above it to 2 (ny - 1) - y; a reflected
    point still outside the range returns the walker to its start."""
    ny, D, seed, N = 6, 4.5, 23, 4000
    n = (5, ny, 4)
    o = orc.Oracle(dict(n=n, bc=("periodic", "wall", "periodic"), tau=0.8, F=(0, 0, 0), D=D, seed=seed))
    rng = np.random.default_rng(2)
    X0 = np.stack([rng.uniform(0, n[0], N), rng.uniform(1.0, ny - 1.0, N), rng.uniform(0, n[2], N)], -1)
    _set_positions(o, X0, n, (2.5, 3.0, 2.0))
    t = o.t
    o.step(1)
    X1 = _unwrapped(*o.walkers(), n)
    z = orc.normals(t, 0, seed, N)
    xf = X0 + math.sqrt(2 * D) * z
    y = xf[:, 1]
    lo, hi = 1.0, ny - 1.0
    yr = np.where(y < lo, 2 * lo - y, np.where(y >= hi, 2 * hi - y, y))
    refl = (y < lo) | (y >= hi)
    back = refl & ((yr < lo) | (yr >= hi))
    exp = xf.copy()
    exp[:, 1] = yr
    exp[back] = X0[back]
    assert back.sum() > 200 and (refl & ~back).sum() > 200
    assert np.max(np.abs(X1 - exp)) < 1e-12
    cn = o.counters()
    assert cn["wall_reflect"] == refl.sum() and cn["returned_to_origin"] == back.sum()
