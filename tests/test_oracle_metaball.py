"""Pins of the oracle's particle geometry: the metaball function (Eq. 3) and
its gradient (Eq. 17), the bounding-radius lemma, the prescribed motion,
Algorithm 1 (binary search for the intersection) and Algorithm 2 (specular
reflection, Eq. 18-22)."""
import math

import numpy as np
import pytest


def _box(n=40):
    return dict(n=(n, n, n), bc=("periodic",) * 3, tau=0.8, F=(0, 0, 0), D=0.0, seed=0)


def _pt(x):
    """continuous position -> (cell, offset)"""
    x = np.asarray(x, float)
    c = np.floor(x)
    return c.astype(np.int32), x - c


def test_single_point_sphere(orc):
    o = orc.Oracle(_box())
    k = 9.0
    c = np.array([20.25, 19.5, 20.75])
    o.add_particle(dict(b=np.zeros((1, 3)), k=np.array([k]), centre=c, motion="static"))
    rng = np.random.default_rng(0)
    for _ in range(200):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        cell, off = _pt(c + math.sqrt(k) * d)
        assert abs(o.particle_M(0, 0, cell, off) - 1.0) < 1e-13
        cell, off = _pt(c + 1.01 * math.sqrt(k) * d)
        assert o.particle_M(0, 0, cell, off) < 1.0
        cell, off = _pt(c + 0.99 * math.sqrt(k) * d)
        assert o.particle_M(0, 0, cell, off) > 1.0


def test_two_point_midplane_ring(orc):
    """Two equal points at +-a along z: on the mid-plane M = 2k/(rho^2 + a^2),
    so M = 1 on the ring rho = sqrt(2k - a^2)."""
    o = orc.Oracle(_box())
    k, a = 5.0, 1.2
    c = np.array([20.0, 20.0, 20.0])
    o.add_particle(dict(b=np.array([[0, 0, a], [0, 0, -a]]), k=np.array([k, k]), centre=c, motion="static"))
    R = math.sqrt(2 * k - a * a)
    for phi in np.linspace(0, 2 * math.pi, 17):
        cell, off = _pt(c + R * np.array([math.cos(phi), math.sin(phi), 0.0]))
        assert abs(o.particle_M(0, 0, cell, off) - 1.0) < 1e-13


def test_gradient_matches_central_differences(orc):
    o = orc.Oracle(_box())
    rng = np.random.default_rng(1)
    b = rng.uniform(-2, 2, size=(6, 3))
    k = rng.uniform(0.3, 1.5, size=6)
    c = np.array([20.0, 20.0, 20.0])
    o.add_particle(dict(b=b, k=k, centre=c, motion="static"))
    h = 1e-5
    for _ in range(50):
        x = c + rng.uniform(-4, 4, size=3)
        cell, off = _pt(x)
        g = o.particle_grad(0, 0, cell, off)
        fd = np.empty(3)
        for ax in range(3):
            e = np.zeros(3)
            e[ax] = h
            fd[ax] = (o.particle_M(0, 0, cell, off + e) - o.particle_M(0, 0, cell, off - e)) / (2 * h)
        assert np.allclose(g, fd, rtol=1e-6, atol=1e-8 * np.abs(g).max())


def test_bounding_radius_lemma(orc):
    o = orc.Oracle(_box(64))
    rng = np.random.default_rng(2)
    b = rng.uniform(-5, 5, size=(10, 3))
    k = rng.uniform(0.3, 1.5, size=10)
    c = np.array([32.0, 32.0, 32.0])
    o.add_particle(dict(b=b, k=k, centre=c, motion="static"))
    rb = o.particle_rb(0)
    assert abs(rb - (np.max(np.linalg.norm(b, axis=1)) + math.sqrt(k.sum()))) < 1e-12
    for _ in range(500):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        cell, off = _pt(c + rb * (1 + 1e-9 + rng.uniform(0, 0.3)) * d)
        assert o.particle_M(0, 0, cell, off) <= 1.0


def test_minimum_image_across_periodic_faces(orc):
    o = orc.Oracle(_box(16))
    o.add_particle(dict(b=np.zeros((1, 3)), k=np.array([4.0]), centre=np.array([0.5, 8.0, 15.5]), motion="static"))
    # (15.0, 8, 0.0) is at distance sqrt(1.5^2 + 0.5^2) from the centre through the faces
    m = o.particle_M(0, 0, np.array([15, 8, 0], np.int32), np.zeros(3))
    assert abs(m - 4.0 / (1.5 ** 2 + 0.5 ** 2)) < 1e-14


def test_sinusoid_pose(orc):
    o = orc.Oracle(_box())
    c0 = np.array([10.0, 11.0, 12.0])
    amp = np.array([4.0, 0.5, 0.0])
    T, ph = 1000.0, 0.37
    o.add_particle(dict(b=np.zeros((1, 3)), k=np.array([1.0]), centre=c0, motion="sinusoid", amp=amp, period=T,
                        phase=ph))
    for t in (0, 1, 250, 999, 1000, 123457):
        c, v = o.particle_pose(0, t)
        arg = 2 * math.pi * (t / T + ph)
        assert np.allclose(c, c0 + amp * math.sin(arg), atol=1e-13)
        assert np.allclose(v, amp * (2 * math.pi / T) * math.cos(arg), atol=1e-15)


def test_algorithm1_against_quadratic(orc):
    """Segment x_p + s (x_f - x_p) through a one-point sphere: the crossing
    s* solves |x_p + s d - c|^2 = k; the bisection result has |M - 1| < 1e-3,
    which bounds |s - s*| by the slope of M along the segment."""
    o = orc.Oracle(_box())
    k = 4.0
    c = np.array([20.0, 20.0, 20.0])
    o.add_particle(dict(b=np.zeros((1, 3)), k=np.array([k]), centre=c, motion="static"))
    rng = np.random.default_rng(3)
    for _ in range(100):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        xp = c + (2.0 + rng.uniform(0.01, 0.5)) * d
        v = d + 0.3 * rng.standard_normal(3)
        xf = c + rng.uniform(0.5, 1.9) * v / np.linalg.norm(v)
        cell, off = _pt(xp)
        dirv = xf - xp
        ok, s = o.bisect(0, 0, cell, off, dirv, 0.0, 1.0)
        assert ok
        x = off + s * dirv
        m = o.particle_M(0, 0, cell, x)
        assert abs(m - 1.0) < 1e-3
        # exact crossing
        p0 = xp - c
        A, B, Cq = dirv @ dirv, 2 * p0 @ dirv, p0 @ p0 - k
        s_star = (-B - math.sqrt(B * B - 4 * A * Cq)) / (2 * A)
        slope = abs(2 * k / 2.0 ** 3 * (dirv @ -(p0 + s_star * dirv)) / 2.0)  # |dM/ds| at the crossing
        assert abs(s - s_star) <= 1.1e-3 / slope + 1e-12


def test_algorithm1_iteration_cap(orc):
    o = orc.Oracle(_box())
    o.add_particle(dict(b=np.zeros((1, 3)), k=np.array([4.0]), centre=np.array([20.0, 20.0, 20.0]),
                        motion="static"))
    cell, off = _pt([23.0, 20.0, 20.0])
    ok, _ = o.bisect(0, 0, cell, off, [-2.9, 0.0, 0.0], 0.0, 1.0, imax=1)
    assert not ok
    ok, s = o.bisect(0, 0, cell, off, [-2.9, 0.0, 0.0], 0.0, 1.0, imax=200)
    assert ok and abs(s - 1.0 / 2.9) < 1e-3


def test_algorithm2_reflection(orc):
    rng = np.random.default_rng(4)
    for _ in range(100):
        ti = rng.standard_normal(3)
        g = rng.standard_normal(3)
        tr = orc.reflect(ti, g)
        n = g / np.linalg.norm(g)
        assert abs(np.linalg.norm(tr) - np.linalg.norm(ti)) < 1e-14
        assert abs(tr @ n + ti @ n) < 1e-14
        # tangential part unchanged
        assert np.allclose(tr - (tr @ n) * n, ti - (ti @ n) * n, atol=1e-14)


def test_reflection_off_sphere_is_specular(orc):
    """For a sphere the gradient at the crossing is radial, so the reflected
    step is the mirror image of the inside part across the tangent plane."""
    c = np.zeros(3)
    x_inter = np.array([0.0, 0.0, 2.0])
    ti = np.array([0.3, 0.1, -0.4])
    g = -2 * 4.0 * (x_inter - c) / np.linalg.norm(x_inter - c) ** 4
    tr = orc.reflect(ti, g)
    assert np.allclose(tr, [0.3, 0.1, 0.4], atol=1e-15)


def test_table1_sphere_projected_area(orc):
    """Table 1 prints A_m = 78.54 for the spherical particle: a sphere of
    radius 5 lattice units (pi 5^2).  The oracle's metaball with one control
    point of weight k = 25 must enclose exactly that disc in its widest
    section (through the centre), counted on a fine grid of the oracle's own
    M >= 1 test (grid error well under 0.5%)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "table1_sphere_projected_area.txt")
    vals = dict(l.split() for l in open(path) if l.strip() and not l.startswith("#"))
    A_m = float(vals["A_m"])
    o = orc.Oracle(_box())
    c = np.array([20.25, 19.5, 20.75])
    o.add_particle(dict(b=np.zeros((1, 3)), k=np.array([25.0]), centre=c, motion="static"))
    h = 0.05
    g = np.arange(-6.0 + h / 2, 6.0, h)
    inside = 0
    for x in g:
        for y in g:
            cell, off = _pt(c + np.array([x, y, 0.0]))
            inside += o.particle_M(0, 0, cell, off) >= 1.0
    area = inside * h * h
    assert abs(area - A_m) / A_m < 5e-3, (area, A_m)
    # a section off the centre is smaller: the widest one is through it
    cell, off = _pt(c + np.array([4.9, 0.0, 1.0]))
    assert o.particle_M(0, 0, cell, off) < 1.0
