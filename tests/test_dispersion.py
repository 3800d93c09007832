"""Pins of the dispersion pipeline (Sec. 4, Eq. 38-40) and of the C ABI's
host-side fit against the oracle's own."""
import math

import numpy as np
import pytest


def test_linear_variance_gives_closed_form_K(orc):
    """sigma^2(t) = a + b t: the slope of Eq. 38 in t is b / (2R)^2 =
    K U_slip / (2R), so K = b / (2R U_slip) and D_alpha = K / (1 - phi)."""
    t = np.linspace(0, 5000, 101)
    a, b, two_r, u_slip, phi = 3.7, 0.0123, 10.0, 0.02, 0.15
    K, Da = orc.dispersion_fit(t, a + b * t, two_r, u_slip, phi)
    assert abs(K - b / (two_r * u_slip)) < 1e-12 * abs(K)
    assert abs(Da - K / (1 - phi)) < 1e-15 * abs(Da)
    # a window starting mid-series sees the same line
    K2, _ = orc.dispersion_fit(t, a + b * t, two_r, u_slip, phi, i0=50)
    assert abs(K2 - K) < 1e-12 * abs(K)


def test_library_fit_matches_oracle(orc):
    from paper_2308_05007_amd import binding as B
    rng = np.random.default_rng(3)
    t = np.sort(rng.uniform(0, 1000, 60))
    s2 = 2.0 + 0.01 * t + 0.3 * rng.standard_normal(60)
    for i0 in (0, 30):
        Ko, Dao = orc.dispersion_fit(t, s2, 10.0, 0.05, 0.2, i0=i0)
        Kl, Dal, off = B.dispersion_fit(t, s2, 10.0, 0.05, 0.2, i0=i0)
        assert abs(Kl - Ko) <= 1e-10 * abs(Ko) and abs(Dal - Dao) <= 1e-10 * abs(Dao)
    with pytest.raises(B.RwmiError):
        B.dispersion_fit(t[:1], s2[:1], 10.0, 0.05, 0.2)


def test_pure_diffusion_variance_grows_as_2Dt(orc):
    """A solute band in a periodic box at rest: sigma_z^2 = sigma_0^2 + 2 D t,
    so with U_slip = 1 and 2R = 1 the fitted K is 2D (within sampling error)."""
    D, n, N = 0.05, 24, 20000
    o = orc.Oracle(dict(n=(n, n, n), bc=("periodic",) * 3, tau=0.8, F=(0, 0, 0), D=D, seed=17))
    assert o.seed(dict(kind="band", band=(2, 11.5, 12.5), ref=(12.0, 12.0, 12.0)), N) == N
    ts, s2 = [], []
    for k in range(11):
        m = o.moments()
        ts.append(m["step"])
        s2.append(m["sumsq"][2] / N - (m["sum"][2] / N) ** 2)
        o.step(10)
    K, _ = orc.dispersion_fit(np.array(ts), np.array(s2), 1.0, 1.0, 0.0)
    # slope standard error ~ 2D sqrt(2/N) relative
    assert abs(K - 2 * D) < 6 * 2 * D * math.sqrt(2.0 / N), (K, 2 * D)
