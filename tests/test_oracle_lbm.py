"""Pins of the oracle's fluid part (Sec. 2.3, Eq. 12-15; bounce-back with the
moving-wall term of Eq. 23; PSM coupling and Guo forcing as readings):
lattice and equilibrium moment invariants, collision invariants, a
brute-force push-stream, and the Poiseuille and Couette closed forms."""
import math

import numpy as np
import pytest

from paper_2308_05007_amd import workloads as W


def test_lattice_moments(orc):
    e, w = orc.lattice()
    assert e.shape == (19, 3)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(w @ e, 0.0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, e, e), np.eye(3) / 3.0, atol=1e-16)
    # third moments vanish, fourth: c_s^4 (d_ab d_cd + d_ac d_bd + d_ad d_bc)
    assert np.allclose(np.einsum("i,ia,ib,ic->abc", w, e, e, e), 0.0, atol=1e-16)
    d = np.eye(3)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, e, e, e, e)
    ref = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.allclose(m4, ref, atol=1e-16)
    # opposite pairs
    for i in range(1, 19):
        j = i + 1 if i % 2 else i - 1
        assert np.array_equal(e[j], -e[i]) and w[i] == w[j]


@pytest.mark.parametrize("rho,u", [(1.0, (0, 0, 0)), (1.07, (0.05, -0.02, 0.01)), (0.93, (-0.1, 0.07, 0.12))])
def test_equilibrium_moments(orc, rho, u):
    e, _ = orc.lattice()
    f = orc.feq(rho, u)
    u = np.asarray(u, float)
    assert abs(f.sum() - rho) < 1e-14
    assert np.allclose(f @ e, rho * u, atol=1e-15)
    assert np.allclose(np.einsum("i,ia,ib->ab", f, e, e), rho * (np.eye(3) / 3 + np.outer(u, u)), atol=1e-14)


def _dom(F=(0, 0, 0), tau=0.8, n=(4, 4, 4), bc=("periodic",) * 3):
    return dict(n=n, bc=bc, tau=tau, F=F, D=0.0, seed=0)


def _random_f(rng, rho=1.0, u=(0.02, -0.01, 0.03), amp=1e-3):
    import oracle
    return oracle.feq(rho, u) * (1.0 + amp * rng.standard_normal(19))


def test_collision_conserves_mass_and_adds_force(orc):
    rng = np.random.default_rng(3)
    e, _ = orc.lattice()
    F = np.array([1e-4, -2e-4, 3e-5])
    o = orc.Oracle(_dom(F=F))
    for eps in (0.0, 0.3, 1.0):
        f = _random_f(rng)
        out, rho, u = o.collide_node(f, eps, [0.01, 0.0, -0.02])
        assert abs(out.sum() - f.sum()) < 1e-15
        if eps == 0.0:
            # Guo: momentum grows by exactly F; u is the half-force velocity
            assert np.allclose(out @ e - f @ e, F, atol=1e-16)
            assert np.allclose(u, (f @ e + F / 2) / f.sum(), atol=1e-17)


def test_psm_solid_limit_and_exchange(orc):
    """B = 1 (eps = 1): the node takes the solid velocity in one step; for any
    eps the change of momentum equals B rho (u_s - u) with F = 0."""
    rng = np.random.default_rng(4)
    e, _ = orc.lattice()
    o = orc.Oracle(_dom(tau=0.7))
    us = np.array([0.03, -0.01, 0.02])
    for eps in (0.0, 0.25, 0.6, 1.0):
        f = _random_f(rng)
        out, rho, u = o.collide_node(f, eps, us)
        B = eps * 0.2 / ((1 - eps) + 0.2)
        dj = out @ e - f @ e
        assert np.allclose(dj, B * rho * (us - u), atol=1e-16)
        if eps == 1.0:
            assert np.allclose((out @ e) / out.sum(), us, atol=1e-16)


def test_eps_zero_ignores_solid_velocity(orc):
    rng = np.random.default_rng(5)
    o = orc.Oracle(_dom(F=(1e-5, 0, 0)))
    f = _random_f(rng)
    a, _, _ = o.collide_node(f, 0.0, [0.0, 0.0, 0.0])
    b, _, _ = o.collide_node(f, 0.0, [0.3, -0.2, 0.1])
    assert np.array_equal(a, b)


def test_tau_one_relaxes_to_equilibrium(orc):
    rng = np.random.default_rng(6)
    o = orc.Oracle(_dom(tau=1.0))
    f = _random_f(rng)
    out, rho, u = o.collide_node(f, 0.0, [0, 0, 0])
    assert np.allclose(out, orc.feq(rho, u), atol=1e-16)


@pytest.mark.parametrize("n,bc", [((4, 5, 6), ("periodic",) * 3), ((5, 4, 3), ("periodic", "wall", "periodic")),
                                  ((7, 5, 6), ("wall", "periodic", "wall"))])
def test_stream_equals_bruteforce_push(orc, n, bc):
    """The oracle's pull-stream equals a push-stream coded independently with
    numpy.roll; the bounce-back populations are checked against the Eq. 23
    form separately (Couette)."""
    rng = np.random.default_rng(7)
    e, w = orc.lattice()
    o = orc.Oracle(_dom(F=(1e-5, 2e-6, 0), tau=0.9, n=n, bc=bc))
    N = int(np.prod(n))
    f0 = np.stack([orc.feq(1.0, (0.01, 0.0, -0.01))] * N, axis=1) * (1 + 1e-3 * rng.standard_normal((19, N)))
    o.set_f(f0)
    # post-collision by the oracle's own node collision
    fs = np.empty_like(f0)
    for k in range(N):
        fs[:, k], _, _ = o.collide_node(f0[:, k], 0.0, [0, 0, 0])
    o.step(1)
    f1 = o.f().reshape(19, -1)
    sh = n[::-1]
    wallm = np.zeros(sh, bool)
    for a in range(3):
        if bc[a] == "wall":
            idx = [slice(None)] * 3
            idx[2 - a] = 0
            wallm[tuple(idx)] = True
            idx[2 - a] = n[a] - 1
            wallm[tuple(idx)] = True
    for i in range(19):
        pushed = np.roll(fs[i].reshape(sh), shift=tuple(int(v) for v in e[i][::-1]), axis=(0, 1, 2))
        src_wall = np.roll(wallm, shift=tuple(int(v) for v in e[i][::-1]), axis=(0, 1, 2))
        m = (~wallm) & (~src_wall)
        assert np.array_equal(f1[i].reshape(sh)[m], pushed[m]), i


def _run_channel(orc, tau, F, ny, steps, wall_lo=None, wall_hi=None):
    dom = dict(n=(1, ny, 1), bc=("periodic", "wall", "periodic"), tau=tau, F=F, D=0.0, seed=0,
               wall_lo=np.zeros(9) if wall_lo is None else wall_lo, wall_hi=np.zeros(9) if wall_hi is None else wall_hi)
    o = orc.Oracle(dom)
    o.step(steps)
    return o.fields()["u"][0, 0, :, 0], o.fields()["rho"][0, :, 0]


def test_poiseuille_magic_tau_is_exact(orc):
    """Plane Poiseuille between halfway walls at y = 1 and y = ny - 1; at
    Lambda = (tau - 1/2)^2 = 3/16 the BGK bounce-back profile is the exact
    parabola u(y) = F/(2 rho nu) (y - 1)(ny - 1 - y), nu = (tau - 1/2)/3."""
    ny, F = 12, 1e-6
    tau = 0.5 + math.sqrt(3.0) / 4.0
    u, rho = _run_channel(orc, tau, (F, 0, 0), ny, 30000)
    nu = (tau - 0.5) / 3.0
    y = np.arange(1, ny - 1) + 0.5
    ref = F / (2 * nu) * (y - 1) * (ny - 1 - y)
    assert np.max(np.abs(u[1:-1] - ref)) / ref.max() < 1e-9


def test_poiseuille_curvature_any_tau(orc):
    """At other tau the interior second difference is -F/(rho nu) exactly and
    only a uniform slip remains."""
    ny, F, tau = 14, 1e-6, 0.8
    u, rho = _run_channel(orc, tau, (F, 0, 0), ny, 40000)
    nu = (tau - 0.5) / 3.0
    d2 = u[1:-3] - 2 * u[2:-2] + u[3:-1]
    assert np.allclose(d2, -F / nu, rtol=1e-8)
    y = np.arange(1, ny - 1) + 0.5
    ref = F / (2 * nu) * (y - 1) * (ny - 1 - y)
    slip = u[1:-1] - ref
    assert np.ptp(slip) < 1e-9 * ref.max()


def test_couette_linear_profile(orc):
    """Walls moving along x with the Eq. 23 term, no force: linear profile
    between the wall velocities at the halfway planes, for any tau."""
    ny, U = 10, 0.01
    wl = np.zeros(9)
    wh = np.zeros(9)
    wl[3] = -U  # lo wall of axis y moves with (-U, 0, 0)
    wh[3] = 2 * U  # hi wall moves with (+2U, 0, 0)
    for tau in (0.6, 1.3):
        u, rho = _run_channel(orc, tau, (0, 0, 0), ny, 30000, wall_lo=wl, wall_hi=wh)
        y = np.arange(1, ny - 1) + 0.5
        ref = -U + 3 * U * (y - 1) / (ny - 2)
        assert np.max(np.abs(u[1:-1] - ref)) < 1e-12
        assert u[0] == -U and u[-1] == 2 * U


def test_mass_conserved_with_moving_particles(orc):
    cfg = W.config_tiny(n=(8, 7, 9), bc=("periodic",) * 3, n_particles=2, n_walkers=0, amp=2.0, spread=1.5)
    o = orc.build_domain(cfg)
    m0 = o.f().sum()
    o.step(30)
    assert abs(o.f().sum() - m0) < 1e-11 * m0
    assert o.fields()["eps"].max() > 0.5


def test_rest_state_stays_at_rest(orc):
    """u0 = 0, F = 0, no particles: every population stays w_i rho0 up to
    rounding and the velocity is exactly zero."""
    o = orc.Oracle(_dom(n=(5, 6, 7)))
    o.step(10)
    _, w = orc.lattice()
    f = o.f().reshape(19, -1)
    assert np.allclose(f, w[:, None], rtol=1e-15, atol=0)
    assert np.all(o.fields()["u"] == 0.0)


def test_solid_fraction_of_one_control_point_sphere(orc):
    """One control point of weight k is a sphere of radius R = sqrt(k), where
    the distance estimate is exact, so eps is the unit ramp 1/2 + (R - r):
    its volume integral is 4/3 pi R^3 + pi R / 3 and the lattice sum must
    match it up to the sampling error of a smooth field."""
    for k, tol in ((4.0, 3e-3), (16.0, 1e-3), (49.0, 5e-4)):
        n = 32
        dom = dict(n=(n, n, n), bc=("periodic",) * 3, tau=0.8, F=(0, 0, 0), D=0.0, seed=0)
        o = orc.Oracle(dom)
        o.add_particle(dict(b=np.zeros((1, 3)), k=np.array([k]), centre=np.array([16.3, 15.8, 16.1]),
                            motion="static"))
        o.step(1)
        eps = o.fields()["eps"]
        R = math.sqrt(k)
        vol = 4.0 / 3.0 * math.pi * R ** 3 + math.pi * R / 3.0
        assert abs(eps.sum() - vol) / vol < tol, (eps.sum(), vol)
        # monotone in M along a ray from the centre
        line = eps[16, 16, 16:]
        assert np.all(np.diff(line) <= 0)


def _two_point_body(orc, k1, k2, a):
    """Oracle eps of a two-control-point metaball (points at +-a on the z axis
    of the particle frame) and the exact signed distance (positive inside) of
    every node centre to the surface M = 1, found without the oracle: the
    body is axisymmetric and star-shaped about its centre, so its meridian
    curve is the root of M = 1 on rays from the centre (bisection), and the
    distance is the nearest point of that curve (dense sampling, refined near
    the surface)."""
    n = 32
    c = np.array([16.3, 15.8, 16.1])
    b = np.array([[0.0, 0.0, -a], [0.0, 0.0, a]])
    kk = np.array([k1, k2])
    o = orc.Oracle(dict(n=(n, n, n), bc=("periodic",) * 3, tau=0.8, F=(0, 0, 0), D=0.0, seed=0))
    o.add_particle(dict(b=b, k=kk, centre=c, motion="static"))
    o.step(1)
    eps = o.fields()["eps"]  # [z, y, x]

    def M(x):
        return sum(kq / np.sum((x - bq) ** 2, -1) for bq, kq in zip(b, kk))

    def meridian(th):
        d = np.stack([np.sin(th), np.zeros_like(th), np.cos(th)], -1)
        lo, hi = np.full_like(th, a * (1 + 1e-9)), np.full_like(th, 4.0 * n)
        for _ in range(52):
            mid = 0.5 * (lo + hi)
            ins = M(mid[:, None] * d) >= 1.0
            lo, hi = np.where(ins, mid, lo), np.where(ins, hi, mid)
        r = 0.5 * (lo + hi)
        return np.stack([r * np.sin(th), r * np.cos(th)], -1)

    th = np.linspace(0.0, math.pi, 2001)
    curve = meridian(th)
    zz, yy, xx = np.meshgrid(*(np.arange(n) + 0.5,) * 3, indexing="ij")
    X = np.stack([xx, yy, zz], -1).reshape(-1, 3) - c
    pts = np.stack([np.hypot(X[:, 0], X[:, 1]), X[:, 2]], -1)
    # nodes farther than 2 from the largest radius of the body lie outside it
    # at a distance of at least 2
    rmax = np.hypot(curve[:, 0], curve[:, 1]).max()
    dist = np.full(len(pts), 2.0)
    near = np.zeros(len(pts), int)
    for s in np.array_split(np.flatnonzero(np.hypot(pts[:, 0], pts[:, 1]) < rmax + 2.0), 16):
        dd = np.hypot(curve[None, :, 0] - pts[s, None, 0], curve[None, :, 1] - pts[s, None, 1])
        near[s] = dd.argmin(1)
        dist[s] = dd.min(1)
    dth = th[1] - th[0]
    # near the surface: ternary search on the ray angle around the nearest sample
    idx = np.flatnonzero(dist < 1.0)
    q = pts[idx]

    def dist_at(t):
        cv = meridian(np.clip(t, 0.0, math.pi))
        return np.hypot(cv[:, 0] - q[:, 0], cv[:, 1] - q[:, 1])

    lo, hi = th[near[idx]] - dth, th[near[idx]] + dth
    for _ in range(40):
        m1, m2 = lo + (hi - lo) / 3, hi - (hi - lo) / 3
        left = dist_at(m1) <= dist_at(m2)
        lo, hi = np.where(left, lo, m1), np.where(left, m2, hi)
    dist[idx] = np.minimum(dist[idx], dist_at(0.5 * (lo + hi)))
    dex = np.where(M(X) >= 1.0, dist, -dist)

    def phi(x):
        return M(x) ** -0.5

    return eps.ravel(), dex, X, phi


def _second_order_bound(phi, X, d):
    """Second-order error bound of a first-order distance estimate on the field
    phi at points X with distance d: |est - d| <= 1/2 ||Hess phi|| d^2 / |grad phi|
    (both by central differences, independent of the oracle)."""
    h = 1e-3
    E = np.eye(3) * h
    g = np.stack([(phi(X + E[i]) - phi(X - E[i])) / (2 * h) for i in range(3)], -1)
    H = np.empty((len(X), 3, 3))
    for i in range(3):
        for j in range(3):
            H[:, i, j] = (phi(X + E[i] + E[j]) - phi(X + E[i] - E[j]) - phi(X - E[i] + E[j]) + phi(X - E[i] - E[j])) / (4 * h * h)
    return 0.5 * np.linalg.norm(H, 2, axis=(1, 2)) * d * d / np.linalg.norm(g, axis=1)


@pytest.mark.parametrize("k1,k2,a", [(36.0, 36.0, 2.0), (36.0, 16.0, 2.5), (25.0, 25.0, 4.0)])
def test_solid_fraction_of_two_point_metaball(orc, k1, k2, a):
    """Beyond one control point the distance in eps = 1/2 + d is a first-order
    estimate (from M^(-1/2), whose level 1 is the surface).  Against the exact
    signed distance it must hold to the second-order bound on every node of
    the ramp (the bound is evaluated at the node; the true error is about a
    third of it at most here, while estimating from M itself, halving the
    distance or flipping its sign each break it on most nodes), and eps must
    be exactly 1 or 0 wherever the exact distance is beyond the ramp.  Unequal
    weights catch a weight paired with the wrong point."""
    eps, dex, X, phi = _two_point_body(orc, k1, k2, a)
    ramp = (eps > 0.0) & (eps < 1.0)
    assert ramp.sum() > 500
    bound = _second_order_bound(phi, X[ramp], dex[ramp])
    err = np.abs((eps[ramp] - 0.5) - dex[ramp])
    assert np.all(err <= bound + 1e-6), (err.max(), bound.max())
    assert np.all(eps[dex > 0.5 + 0.02] == 1.0)
    assert np.all(eps[dex < -0.5 - 0.02] == 0.0)
