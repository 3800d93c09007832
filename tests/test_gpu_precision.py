"""Precision modes (distributions stored as deviations in FP32 / FP16 /
BF16, float collision and walkers) against the FP64 GPU mode on a reduced
oscillator (64^3, 8 metaballs, 1e5 walkers in a band, 500 steps).  The bounds
are ten times the measured errors of this case; the full 256^3 comparison is
bench.py --workload precision."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

BOUNDS = {  # velocity L2, concentration L2, D_alpha relative, 99th pct position error (cells)
    "fp32": (5e-5, 0.02, 1e-5, 2e-5),
    "fp16": (3e-3, 0.04, 1e-4, 3e-4),
    "bf16": (1.5e-2, 0.06, 2e-3, 3e-3),
}


@pytest.fixture(scope="module")
def report():
    from paper_2308_05007_amd import precision, workloads as W
    cfg = W.config_oscillator(n=64, n_particles=8, n_walkers=100_000, steps=500)
    return precision.report(cfg, steps=500, every=5)


@pytest.mark.parametrize("mode", ["fp32", "fp16", "bf16"])
def test_mode_within_stated_bounds(report, mode):
    r = report[mode]
    bv, bc, bd, bp = BOUNDS[mode]
    assert r["velocity_l2"] < bv, r
    assert r["concentration_l2"] < bc, r
    assert r["D_alpha_rel"] < bd, r
    assert r["pos_p99"] < bp, r


def test_dispersion_coefficient_is_positive_and_finite(report):
    f = report["fp64"]
    assert np.isfinite(f["D_alpha"]) and f["D_alpha"] > 0 and f["u_slip"] > 0
