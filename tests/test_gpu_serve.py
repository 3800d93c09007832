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


def test_served_fp64_requests_match_oracle():
    """FP64 requests through the continuous-batching server (staggered
    arrivals, mixed with each other, retired at different times): the moments
    each served request reports equal its oracle run (walker count and event
    counters exactly, sums within the recursive-summation bound of the sum of
    the absolute values of their terms)."""
    import oracle
    from paper_2308_05007_amd import serve, workloads as W
    rng = np.random.default_rng(41)
    reqs = []
    for i in range(5):
        r = W.serving_request(i, rng, steps_range=(12, 30), edges=(16, 24, 32), walker_range=(500, 4000),
                              particle_range=(1, 3), precisions=("fp64",))
        reqs.append(r)
    trace = [(0.0, reqs[0]), (0.0, reqs[1]), (0.02, reqs[2]), (0.05, reqs[3]), (0.05, reqs[4])]
    st, _ = serve.run_continuous(trace, budget_bytes=8 << 30, chunk=5, keep_results=True)
    assert sorted(st.results) == list(range(len(trace)))
    for rid, (_, req) in enumerate(trace):
        o = oracle.build_domain(req)
        w = req["walkers"]
        assert o.seed(w, w["n"]) == w["n"]
        o.step(req["steps"])
        mo = o.moments()
        got = st.results[rid]
        assert got["step"] == req["steps"] and got["n_walkers"] == w["n"]
        assert got["counters"] == o.counters()
        cell, off, img = o.walkers()
        n = np.asarray(req["domain"]["n"])
        X = np.stack([cell % n[0], (cell // n[0]) % n[1], cell // (n[0] * n[1])]) + img * n[:, None] + off
        dx = X - o.ref()[:, None]
        # recursive-summation bound: gamma_k sum |x_i|, k the longest chain of
        # additions of either side (the oracle's, one after another)
        gam = lambda k: k * 2.0 ** -53 / (1 - k * 2.0 ** -53)
        nw_, nn = w["n"], int(np.prod(n))
        for k, scale in (("sum", np.abs(dx).sum(1)), ("sumsq", (dx * dx).sum(1))):
            err = np.abs(np.asarray(got[k]) - mo[k])
            assert np.all(err <= gam(nw_ + 4098) * scale), (rid, k, err, scale)
        assert abs(got["mass"] - mo["mass"]) <= gam(nn + 4098) * abs(mo["mass"])
