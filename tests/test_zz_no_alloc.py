"""The allocation-free moment read-out (rwmi_read_moments_noalloc) against the
allocating one (rwmi_read_moments), through the C ABI: the same kernels and
reduction order, so the moments must be identical bit for bit.  Two calls in
a row on domains of decreasing size (stale partials of the first call lie in
the scratch array beyond what the second uses), then a domain too large for
the scratch array, which must be refused with EINVAL."""
import ctypes as C

import numpy as np
import pytest

from paper_2308_05007_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2308_05007_amd import binding
    binding.lib()
    return binding


def _same(a, b):
    for k in ("step", "n_walkers", "mass", "solid_volume", "near_surface"):
        assert a[k] == b[k], k
    for k in ("sum", "sumsq", "momentum", "fluid_u", "particle_v"):
        assert np.array_equal(a[k], b[k]), (k, a[k], b[k])
    assert a["counters"] == b["counters"]


def _run(B, cfg, steps):
    g = B.build_domain(cfg)
    g.step(steps)
    ref = g.moments()
    got = g.moments(noalloc=True)
    return g, ref, got


def test_noalloc_moments_equal_allocating_read_twice(B):
    big = W.config_oscillator(precision="fp32", n=96, n_particles=12, n_walkers=300_000, steps=40)
    small = W.config_tiny(n=(17, 9, 11), bc=("periodic", "wall", "periodic"), n_particles=2, n_walkers=700,
                          seed=13, precision="fp64")
    g1, r1, a1 = _run(B, big, 12)
    assert r1["n_walkers"] == 300_000 and r1["solid_volume"] > 0
    _same(a1, r1)
    g2, r2, a2 = _run(B, small, 9)
    _same(a2, r2)
    # and once more on the first domain after stepping it further
    g1.step(5)
    _same(g1.moments(noalloc=True), g1.moments())
    g1.close()
    g2.close()


def test_noalloc_moments_refuse_a_lattice_beyond_the_scratch(B):
    # 64 + 12 ceil(N / 4096) > 131072 for N = 360^3
    dom = dict(n=(360, 360, 360), bc=("periodic",) * 3, tau=0.8, F=(0, 0, 0), D=0.0, seed=0, precision="fp16")
    g = B.Domain(dom)
    m = B.Moments()
    st = g.L.rwmi_read_moments_noalloc(g.h, C.byref(m))
    assert st == B.RWMI_EINVAL
    assert "allocation-free" in g.L.rwmi_last_error(g.h).decode()
    g.close()
