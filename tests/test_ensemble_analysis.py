"""Pins of the host-side analysis of the shape sweep (Sec. 4, Eq. 38-45):
the Gaussian fit of a concentration profile (library and oracle), the shape
features of Eq. 41-44 against closed forms for spheres and ellipsoids
(Table 1's sphere among them), the Spearman correlation of Eq. 45 against
scipy and against the correlations the paper reads off its Table 1, and the
oracle's concentration profile against its occupancy."""
import math
import os

import numpy as np
import pytest
from scipy import special, stats
from scipy.optimize import curve_fit

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_shape_features.txt")


def _gauss(x, a, m, v):
    return a * np.exp(-(x - m) ** 2 / (2 * v))


@pytest.mark.parametrize("impl", ["oracle", "library"])
def test_gaussian_fit_exact_and_noisy(orc, impl):
    from paper_2308_05007_amd import binding as B
    fit = orc.gaussian_fit if impl == "oracle" else B.gaussian_fit
    x = np.arange(80) + 0.5
    for a, m, v in ((3.7, 17.3, 4.2), (1e6, 40.0, 90.0), (25.0, 60.2, 0.8)):
        got = fit(x, _gauss(x, a, m, v))
        assert np.allclose(got, (a, m, v), rtol=1e-9, atol=1e-9), got
    rng = np.random.default_rng(2)
    y = _gauss(x, 1000.0, 39.7, 31.0) + rng.normal(0, 8.0, x.size)
    ref = curve_fit(_gauss, x, y, p0=(900, 40, 25), xtol=1e-14, ftol=1e-14)[0]
    assert np.allclose(fit(x, y), ref, rtol=1e-7)


def test_gaussian_fit_needs_three_positive_points(orc):
    from paper_2308_05007_amd import binding as B
    x = np.arange(20) + 0.5
    y = np.zeros(20)
    y[[9, 10]] = (40.0, 60.0)
    with pytest.raises(ValueError):
        orc.gaussian_fit(x, y)
    with pytest.raises(B.RwmiError):
        B.gaussian_fit(x, y)
    y[11] = 1.0
    assert np.allclose(B.gaussian_fit(x, y), orc.gaussian_fit(x, y), rtol=1e-9)


def test_gaussian_fit_library_equals_oracle(orc):
    from paper_2308_05007_amd import binding as B
    rng = np.random.default_rng(5)
    x = np.arange(120) + 0.5
    for _ in range(5):
        y = np.maximum(0, _gauss(x, rng.uniform(10, 1e5), rng.uniform(40, 80), rng.uniform(2, 200))
                       + rng.normal(0, 1.0, x.size)).round()
        assert np.allclose(B.gaussian_fit(x, y), orc.gaussian_fit(x, y), rtol=1e-9)


def test_sphere_features_and_table1_area():
    """A one-point metaball of weight 25 is the sphere of radius 5 of Table 1:
    every feature is 1 and A_m = 78.54 (pi R^2); volume and area are the
    sphere's to second order in the grid spacing."""
    from paper_2308_05007_amd import shapes as S
    f = S.features(S.Metaball(np.zeros((1, 3)), [25.0]), h=0.15, n_dirs=6)
    am = float(open(GOLDEN).read().split("Sphere")[1].split()[4])
    assert abs(f["A_m"] - am) < 0.005 * am
    assert abs(f["volume"] - 4 / 3 * math.pi * 125) < 0.003 * 523.6
    assert abs(f["area"] - 4 * math.pi * 25) < 0.005 * 314.2
    for k in ("sphericity", "C_c", "D_ns", "CSF"):
        assert abs(f[k] - 1.0) < 0.006, (k, f[k])


def _ellipsoid_area(a, b, c):
    """Surface area of an ellipsoid a >= b >= c (Legendre's form with the
    incomplete elliptic integrals)."""
    phi = math.acos(c / a)
    k2 = a * a * (b * b - c * c) / (b * b * (a * a - c * c))
    E, F = special.ellipeinc(phi, k2), special.ellipkinc(phi, k2)
    return 2 * math.pi * c * c + 2 * math.pi * a * b / math.sin(phi) * (E * math.sin(phi) ** 2 + F * math.cos(phi) ** 2)


def test_ellipsoid_features_closed_forms():
    """Ellipsoid of semi-axes 6, 4, 3, randomly rotated: volume 4/3 pi abc,
    surface area (elliptic integrals), largest projection the ellipse pi a b
    with Ramanujan's perimeter, principal extents 2c, 2b, 2a, CSF c/sqrt(ab)."""
    from paper_2308_05007_amd import shapes as S
    from paper_2308_05007_amd.workloads import _rotation
    a, b, c = 6.0, 4.0, 3.0
    body = S.Ellipsoid(a, b, c).rotated(_rotation(np.random.default_rng(4)))
    f = S.features(body, h=0.15, n_dirs=24)
    assert abs(f["volume"] - 4 / 3 * math.pi * a * b * c) < 0.003 * f["volume"]
    A = _ellipsoid_area(a, b, c)
    assert abs(f["area"] - A) < 0.006 * A
    assert abs(f["A_m"] - math.pi * a * b) < 0.01 * math.pi * a * b
    hh = ((a - b) / (a + b)) ** 2
    P = math.pi * (a + b) * (1 + 3 * hh / (10 + math.sqrt(4 - 3 * hh)))
    assert abs(f["P_p"] - P) < 0.01 * P
    assert np.allclose(f["axes"], (2 * c, 2 * b, 2 * a), rtol=0.01)
    assert abs(f["CSF"] - c / math.sqrt(a * b)) < 0.01
    Dn = (6 * 4 / 3 * math.pi * a * b * c / math.pi) ** (1 / 3)
    assert abs(f["D_ns"] - Dn / math.sqrt(4 * a * b)) < 0.01
    assert abs(f["sphericity"] - math.pi * Dn * Dn / A) < 0.01


def test_metaball_scaling_is_exact():
    """Offsets x s and weights x s^2 scale a metaball by s: its volume by s^3."""
    from paper_2308_05007_amd import shapes as S, workloads as W
    b, k = W.ensemble_base_shapes()["D"]
    m = S.Metaball(b, k)
    v1 = S.volume_area(m, m.radius / 30)[0]
    v2 = S.volume_area(m.scaled(2.5), 2.5 * m.radius / 30)[0]
    assert abs(v2 - 2.5 ** 3 * v1) < 1e-9 * v2


def test_spearman_against_scipy_and_eq45():
    from paper_2308_05007_amd import shapes as S
    rng = np.random.default_rng(7)
    for n in (3, 5, 12, 50):
        x = rng.integers(0, 6, n).astype(float)  # with ties
        y = x * rng.uniform(0.5, 2, n) + rng.normal(0, 1, n)
        assert abs(S.spearman(x, y) - stats.spearmanr(x, y)[0]) < 1e-12
        u = rng.permutation(n).astype(float)
        v = rng.permutation(n).astype(float)
        d2 = ((S.ranks(u) - S.ranks(v)) ** 2).sum()
        assert abs(S.spearman(u, v) - (1 - 6 * d2 / (n * (n * n - 1)))) < 1e-12


def test_table1_correlations():
    """The correlations the paper reads off Table 1 (Fig. 20): A_m is
    negatively correlated with the other features, which are positively
    correlated among themselves; C_c has the strongest association with
    D_alpha and CSF the weakest."""
    from paper_2308_05007_amd import shapes as S
    rows = [ln.split() for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    cols = {k: [float(r[i]) for r in rows] for i, k in enumerate(("phi", "C_c", "D_ns", "CSF", "A_m", "D_alpha"), 1)}
    m = S.spearman_matrix(cols)
    feats = ("phi", "C_c", "D_ns", "CSF")
    assert all(m["A_m"][f] < -0.6 for f in feats)
    assert all(m[f][g] > 0.5 for f in feats for g in feats)
    assoc = {f: abs(m[f]["D_alpha"]) for f in feats + ("A_m",)}
    assert max(assoc, key=assoc.get) == "C_c"
    assert assoc["CSF"] == min(assoc.values())


def test_oracle_profile_is_occupancy_summed(orc):
    from paper_2308_05007_amd import workloads as W
    cfg = W.config_tiny(n=(7, 9, 11), bc=("periodic", "wall", "periodic"), n_particles=2, n_walkers=900, seed=3)
    o = orc.build_domain(cfg)
    o.seed(cfg["walkers"], 900)
    o.step(4)
    occ = o.occupancy()  # [z][y][x]
    for axis, red in ((0, (0, 1)), (1, (0, 2)), (2, (1, 2))):
        assert np.array_equal(o.profile(axis), occ.sum(axis=red).astype(np.uint64))
    assert int(o.profile(2).sum()) == 900
