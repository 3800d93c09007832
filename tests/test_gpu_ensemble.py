"""The shape sweep of Sec. 4 on the GPU: the concentration-profile kernel
against the oracle (exact counts, both the block-histogram and the global
path), and a small FP64 sweep (two shapes, two realisations each, one batch)
whose realisation-averaged profiles, velocity averages, Gaussian-fit
variances, K and D_alpha equal those of the same realisations run by the
oracle."""
import numpy as np
import pytest

from paper_2308_05007_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2308_05007_amd import binding
    binding.lib()
    return binding


@pytest.mark.parametrize("n", [(13, 9, 21), (4200, 3, 2)])
def test_profile_matches_oracle(orc, B, n):
    cfg = W.config_tiny(n=n, bc=("periodic",) * 3, n_particles=1, n_walkers=5000, seed=9, D=0.3, spread=0.6)
    o = orc.build_domain(cfg)
    g = B.build_domain(cfg, seed_walkers=False)
    w = cfg["walkers"]
    assert o.seed(w, w["n"]) == g.seed(w, w["n"]) == w["n"]
    for steps in (0, 7):
        o.step(steps)
        g.step(steps)
        for axis in range(3):
            assert np.array_equal(g.profile(axis), o.profile(axis)), (n, axis)


def test_small_fp64_sweep_matches_oracle(orc, B):
    from paper_2308_05007_amd import ensemble as E
    shapes = E.equal_volume_shapes(R=1.5, h=0.05)
    shapes = {k: shapes[k] for k in ("sphere", "B")}
    kw = dict(realisations=2, steps=60, every=10, R=1.5, n_particles=5, n_walkers=4000, D=0.02, precision="fp64")
    res, ser, perf = E.run(shapes, **kw)
    nz = int(round(36 * 1.5))
    z = np.arange(nz) + 0.5
    for si, name in enumerate(shapes):
        body = shapes[name]
        os_ = []
        for r in range(2):
            cfg = W.config_ensemble_member(name, body.b, body.k, r, shape_index=si, R=1.5, n_particles=5,
                                           n_walkers=4000, steps=60, D=0.02, precision="fp64")
            o = orc.build_domain(cfg)
            assert o.seed(cfg["walkers"], 4000) == 4000
            os_.append(o)
        prof, fu, pv, sol, ts = [], [], [], [], []
        for k in range(7):
            prof.append(sum(o.profile(2).astype(float) for o in os_) / 2)
            ms = [o.moments() for o in os_]
            fu.append(sum(m["fluid_u"] for m in ms) / 2)
            pv.append(sum(m["particle_v"] for m in ms) / 2)
            sol.append(sum(m["solid_volume"] for m in ms) / 2)
            ts.append(10 * k)
            if k < 6:
                for o in os_:
                    o.step(10)
        s = ser[name]
        for k in range(7):
            assert np.array_equal(s["profile"][k], prof[k]), (name, k)
            assert np.allclose(s["fluid_u"][k], fu[k], rtol=1e-9, atol=1e-15)
            assert np.allclose(s["particle_v"][k], pv[k], rtol=1e-9, atol=1e-15)
            assert abs(s["solid"][k] - sol[k]) <= 1e-9 * max(abs(sol[k]), 1.0)
        sig2 = np.array([orc.gaussian_fit(z, p)[2] if np.count_nonzero(p) >= 3 else np.nan for p in prof])
        assert np.allclose(res[name]["sigma2"], sig2, rtol=1e-8, equal_nan=True)
        fux, pvx = np.array(fu)[:, 0], np.array(pv)[:, 0]
        u_slip = abs(fux.max() - pvx.max())
        phi = np.mean(sol[1:]) / float(np.prod(cfg["domain"]["n"]))
        K, Da = orc.dispersion_fit(np.array(ts, float), sig2, 3.0, u_slip, phi, i0=3)
        assert abs(res[name]["K"] - K) <= 1e-6 * abs(K) and abs(res[name]["D_alpha"] - Da) <= 1e-6 * abs(Da)
