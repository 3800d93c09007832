"""Host logic of the serving loop without a GPU: the Poisson trace and the
footprint-based admission arithmetic."""
import numpy as np


def test_poisson_trace_rate_and_order():
    from paper_2308_05007_amd import workloads as W
    tr = W.serving_trace(rate=20.0, duration=10.0, seed=5)
    t = np.array([a for a, _ in tr])
    assert np.all(np.diff(t) > 0) and t[-1] <= 10.0
    # 200 expected arrivals, Poisson sd ~ 14.1
    assert abs(len(tr) - 200) < 5 * 14.2
    gaps = np.diff(t)
    assert abs(gaps.mean() - 0.05) < 0.015
    r = tr[0][1]
    assert r["domain"]["precision"] in ("fp32", "fp16") and 500 <= r["steps"] <= 3000
    assert 32 <= r["domain"]["n"][0] <= 128 and 1e4 <= r["walkers"]["n"] <= 1e6


def test_footprint_orders_requests():
    from paper_2308_05007_amd import serve, workloads as W
    rng = np.random.default_rng(1)
    reqs = [W.serving_request(i, rng) for i in range(8)]
    fps = [serve.footprint(r) for r in reqs]
    nodes = [serve.nodes_of(r) for r in reqs]
    # the distributions dominate: footprint grows with the lattice
    assert np.corrcoef(fps, nodes)[0, 1] > 0.9
