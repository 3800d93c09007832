"""Serving: results of requests run through the continuous-batching server
(admitted at different times, mixed with others, retired at different times)
are bit-identical to the same requests run alone."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _small_trace():
    from paper_2308_05007_amd import workloads as W
    rng = np.random.default_rng(21)
    reqs = [W.serving_request(i, rng, steps_range=(30, 90), edges=(16, 24, 32), walker_range=(500, 5000),
                              particle_range=(2, 4)) for i in range(6)]
    # staggered arrivals: the first ones run alone for a while, later ones join
    return [(0.0, reqs[0]), (0.0, reqs[1]), (0.05, reqs[2]), (0.1, reqs[3]), (0.3, reqs[4]), (0.3, reqs[5])]


def test_served_equals_alone():
    from paper_2308_05007_amd import serve
    trace = _small_trace()
    alone, _ = serve.run_fifo(trace, keep_results=True)
    mixed, _ = serve.run_continuous(trace, budget_bytes=8 << 30, chunk=7, keep_results=True)
    static, _ = serve.run_static(trace, batch_size=3, keep_results=True)
    assert sorted(alone.results) == sorted(mixed.results) == sorted(static.results) == list(range(len(trace)))
    for rid, r in alone.results.items():
        assert mixed.results[rid] == r, rid
        assert static.results[rid] == r, rid


def test_admission_respects_budget():
    from paper_2308_05007_amd import serve
    trace = _small_trace()
    fps = [serve.footprint(r) for _, r in trace]
    # room for the two largest at most: requests must wait for memory
    budget = sorted(fps)[-1] + sorted(fps)[-2]
    st, _ = serve.run_continuous(trace, budget_bytes=budget, chunk=5)
    assert len(st.lat) == len(trace)
