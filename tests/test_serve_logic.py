"""Host logic of the serving loop without a GPU: the Poisson trace, the
footprint-based admission arithmetic, and the continuous-batching, static
and FIFO loops driven by a fake executor on a seeded virtual clock (a cost
model stands in for the device): admission by footprint and free slots in
arrival order, no newcomer in a running static batch, and the latency
percentiles."""
import numpy as np
import pytest


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


# ------------------------------------------------------------------ fake device
class FakeDomain:
    def __init__(self, req):
        self.req = req
        self.steps = 0
        self.alive = True
        self.batch = None


class FakeBatch:
    def __init__(self):
        self.members = []
        self.closed = False


class FakeExecutor:
    """A cost model of the device on a virtual clock: a launch group of n steps
    over domains of N nodes in all takes n (t0 + N / (R min(1, N / N_fill)))
    seconds, so that a lattice too small to fill the GPU runs at the rate of
    N_fill nodes.  Footprint: 168 bytes per node and 20 per walker.  Every
    batch membership and lifetime rule of the library is asserted."""

    def __init__(self, clock, R=3e10, N_fill=4e6, t0=5e-6, budget=None, max_slots=None):
        self.clock, self.R, self.N_fill, self.t0 = clock, R, N_fill, t0
        self.budget, self.max_slots = budget, max_slots
        self.live = set()
        self.work_log = []

    def footprint(self, req):
        return 168 * int(np.prod(req["domain"]["n"])) + 20 * req["walkers"]["n"]

    def _cost(self, nodes, n):
        return n * (self.t0 + nodes / (self.R * min(1.0, nodes / self.N_fill)))

    def create(self, req):
        d = FakeDomain(req)
        self.live.add(id(d))
        return d

    def run_alone(self, d, steps):
        assert d.alive and d.batch is None
        self.clock.advance(self._cost(int(np.prod(d.req["domain"]["n"])), steps))
        d.steps += steps

    def result(self, d):
        assert d.alive
        return {"step": d.steps, "name": d.req["name"]}

    def destroy(self, d):
        assert d.alive and d.batch is None, "a domain is destroyed only after leaving its batch"
        d.alive = False
        self.live.discard(id(d))

    def new_batch(self, use_graph=True, launch=None):
        return FakeBatch()

    def batch_add(self, bt, d):
        assert d.alive and d.batch is None and not bt.closed
        bt.members.append(d)
        d.batch = bt
        if self.budget is not None:
            assert sum(self.footprint(m.req) for m in bt.members) <= self.budget
        if self.max_slots is not None:
            assert len(bt.members) <= self.max_slots

    def batch_remove(self, bt, d):
        assert d in bt.members
        bt.members.remove(d)
        d.batch = None

    def batch_step(self, bt, n):
        assert bt.members and all(m.alive for m in bt.members)
        nodes = sum(int(np.prod(m.req["domain"]["n"])) for m in bt.members)
        for m in bt.members:
            assert m.steps + n <= m.req["steps"], "a request is never stepped past its end"
            m.steps += n
        self.work_log.append((self.clock.now(), len(bt.members), n))
        self.clock.advance(self._cost(nodes, n))

    def batch_close(self, bt):
        assert not bt.members
        bt.closed = True


def _trace(rate, duration, seed, steps=(200, 600)):
    from paper_2308_05007_amd import workloads as W
    return W.serving_trace(rate=rate, duration=duration, seed=seed, steps_range=steps)


def _run(mode, trace, **kw):
    from paper_2308_05007_amd import serve
    clk = serve.VirtualClock()
    ex = FakeExecutor(clk, budget=kw.get("budget_bytes"), max_slots=kw.get("max_slots"))
    if mode == "continuous":
        st, wall = serve.run_continuous(trace, kw["budget_bytes"], max_slots=kw.get("max_slots", 64),
                                        chunk=kw.get("chunk", 50), keep_results=True, executor=ex, clock=clk)
    elif mode == "static":
        st, wall = serve.run_static(trace, batch_size=kw.get("batch_size", 16), keep_results=True, executor=ex,
                                    clock=clk)
    else:
        st, wall = serve.run_fifo(trace, keep_results=True, executor=ex, clock=clk)
    assert not ex.live, "every domain is destroyed"
    return st, wall, ex


def test_every_request_completes_with_its_own_step_count():
    trace = _trace(20.0, 3.0, 7)
    for mode in ("continuous", "static", "fifo"):
        st, wall, ex = _run(mode, trace, budget_bytes=8 << 30)
        assert sorted(st.results) == list(range(len(trace)))
        for rid, (_, req) in enumerate(trace):
            assert st.results[rid] == {"step": req["steps"], "name": req["name"]}
        assert len(st.lat) == len(trace) and min(st.lat) > 0


def test_admission_by_footprint_and_slots_in_arrival_order():
    """A budget of three average requests and four slots: the server never
    holds more (asserted inside the fake executor at every admission),
    requests wait in the queue, and they are admitted in arrival order."""
    from paper_2308_05007_amd import serve
    trace = _trace(40.0, 2.0, 11)
    fx = FakeExecutor(serve.VirtualClock())
    fps = [fx.footprint(r) for _, r in trace]
    budget = max(max(fps), 3 * int(np.mean(fps)))
    st, wall, ex = _run("continuous", trace, budget_bytes=budget, max_slots=4, chunk=25)
    admits = [rid for ev, rid, _ in st.trace_log if ev == "admit"]
    assert admits == sorted(admits) == list(range(len(trace)))
    assert st.max_queue > 1 and st.peak_slots <= 4 and st.peak_used <= budget
    assert max(m for _, m, _ in ex.work_log) <= 4


def test_requests_join_a_running_batch():
    """Continuous batching: a request that arrives while others are on the
    device is admitted at the next chunk boundary and steps together with
    them (the batch holds more than one member at some point, and members
    are admitted while others are part-way through)."""
    trace = _trace(20.0, 2.0, 3)
    st, wall, ex = _run("continuous", trace, budget_bytes=8 << 30, chunk=20)
    assert max(m for _, m, _ in ex.work_log) > 1
    t_admit = {rid: t for ev, rid, t in st.trace_log if ev == "admit"}
    t_done = {rid: t for ev, rid, t in st.trace_log if ev == "done"}
    overlaps = sum(1 for a in t_admit for b in t_admit if a != b and t_admit[a] < t_admit[b] < t_done[a])
    assert overlaps > 0


def test_static_batches_admit_nobody_while_running():
    trace = _trace(20.0, 2.0, 5)
    st, wall, ex = _run("static", trace, batch_size=4)
    events = sorted(st.trace_log, key=lambda e: e[2])
    # a batch is admitted as a whole, then only completions follow until it is empty
    live = set()
    admitting = True
    for ev, rid, t in events:
        if ev == "admit":
            assert admitting or not live, "admitted %d into a running static batch" % rid
            live.add(rid)
        else:
            admitting = False
            live.discard(rid)
            if not live:
                admitting = True


def test_percentiles():
    from paper_2308_05007_amd import serve
    rng = np.random.default_rng(2)
    for n in (1, 2, 7, 100, 1001):
        x = rng.exponential(size=n)
        for q in (50, 90, 99):
            assert abs(serve.percentile(x, q) - np.percentile(x, q)) < 1e-12
    assert serve.percentile([3.0, 1.0, 2.0], 50) == 2.0


def test_latencies_on_a_hand_computed_trace():
    """Three requests of one size arriving together, each taking exactly 1 s
    alone on the cost model: FIFO completes them at 1, 2 and 3 s (p50 2 s,
    p99 2.98 s); the continuous server steps them together and finishes all
    three when the shared batch does."""
    from paper_2308_05007_amd import serve, workloads as W
    rng = np.random.default_rng(0)
    req = W.serving_request(0, rng, steps_range=(100, 100), edges=(128,), particle_range=(2, 2))
    trace = [(0.0, dict(req, name="a")), (0.0, dict(req, name="b")), (0.0, dict(req, name="c"))]
    clk = serve.VirtualClock()
    ex = FakeExecutor(clk, t0=0.0, N_fill=1.0)
    N = int(np.prod(req["domain"]["n"]))
    ex.R = N * 100 / 1.0  # 100 steps of one request in 1 s
    st, wall = serve.run_fifo(trace, executor=ex, clock=clk)
    assert np.allclose(sorted(st.lat), [1.0, 2.0, 3.0])
    s = st.summary(wall)
    assert abs(s["p50_s"] - 2.0) < 1e-12 and abs(s["p99_s"] - 2.98) < 1e-12
    clk = serve.VirtualClock()
    ex = FakeExecutor(clk, t0=0.0, N_fill=1.0)
    ex.R = N * 100 / 1.0
    st, wall = serve.run_continuous(trace, 8 << 30, chunk=30, executor=ex, clock=clk)
    assert np.allclose(st.lat, [3.0, 3.0, 3.0])


def test_continuous_batching_beats_fifo_under_load():
    """Requests far smaller than the GPU: stepped together they fill it, one at
    a time they do not, so under load the continuous server's p99 latency and
    throughput are better than FIFO's on the same trace."""
    trace = _trace(20.0, 5.0, 9, steps=(500, 1500))
    c, wc, _ = _run("continuous", trace, budget_bytes=64 << 30)
    f, wf, _ = _run("fifo", trace)
    sc, sf = c.summary(wc), f.summary(wf)
    assert sc["p99_s"] < sf["p99_s"] and sc["MLUPS"] > sf["MLUPS"]
