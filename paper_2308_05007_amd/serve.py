"""Serving: a request loop over a Poisson stream of independent solves.

Continuous batching (`run_continuous`): every request is a domain whose state
stays in HBM from admission to completion.  At each chunk boundary the
server admits queued requests in arrival order while their device footprint
(rwmi_footprint_bytes) fits the memory budget and a slot is free, steps all
admitted domains together (one rwmi batch: every kernel of a step is one
launch over all members), and retires the ones that reached their step count
(reads their moments, frees their memory).  Requests that arrive while others
run therefore start as soon as memory and a slot free up, and their work
overlaps on the device.

Baselines on the same trace: `run_fifo` runs each request alone, one after
the other; `run_static` waits for a batch of requests, runs the batch to
completion without admitting newcomers, then forms the next.

Latency is measured from arrival to completion on the loop's clock.  A
request's result does not depend on what else is in the batch (same
arithmetic per node and per walker).

The loops drive an executor (`GpuExecutor`: the library through the binding)
and read a clock (`WallClock`).  Tests drive the same loops with a cost model
on a virtual clock (`VirtualClock` and a fake executor), which checks the
admission, slot and latency logic without a GPU.
"""
import json
import time

import numpy as np

from . import binding as B
from . import workloads as W


def footprint(req):
    parts = req["particles"]
    return B.footprint_bytes(req["domain"], len(parts), sum(len(p["k"]) for p in parts), req["walkers"]["n"])


def nodes_of(req):
    return int(np.prod(req["domain"]["n"]))


def percentile(x, q):
    """The q-th percentile of x by linear interpolation between order
    statistics (position q/100 (n - 1) in the sorted sample)."""
    x = np.sort(np.asarray(x, float))
    if x.size == 0:
        return float("nan")
    pos = q / 100.0 * (x.size - 1)
    lo = int(np.floor(pos))
    hi = min(lo + 1, x.size - 1)
    return float(x[lo] + (pos - lo) * (x[hi] - x[lo]))


class Stats:
    def __init__(self):
        self.lat = []
        self.node_steps = 0
        self.walker_steps = 0
        self.max_queue = 0
        self.results = {}
        self.trace_log = []  # (event, rid, time)

    def done(self, rid, req, arrival, now, result=None):
        self.lat.append(now - arrival)
        self.node_steps += nodes_of(req) * req["steps"]
        self.walker_steps += req["walkers"]["n"] * req["steps"]
        self.trace_log.append(("done", rid, now))
        if result is not None:
            self.results[rid] = result

    def summary(self, wall):
        lat = self.lat if self.lat else [float("nan")]
        return {"completed": len(self.lat), "p50_s": percentile(lat, 50), "p99_s": percentile(lat, 99),
                "mean_s": float(np.mean(lat)), "wall_s": wall, "MLUPS": self.node_steps / wall / 1e6,
                "walker_steps_per_s": self.walker_steps / wall, "max_queue": self.max_queue}


class WallClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0

    def sleep(self, dt):
        if dt > 0:
            time.sleep(dt)


class VirtualClock:
    """A clock that only moves when told to (by sleeps and by the fake
    executor's work)."""

    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep(self, dt):
        if dt > 0:
            self.t += dt

    def advance(self, dt):
        self.t += dt


def _result(d):
    m = d.moments()
    return {"step": m["step"], "n_walkers": m["n_walkers"], "sum": m["sum"].tolist(), "sumsq": m["sumsq"].tolist(),
            "mass": m["mass"], "counters": m["counters"]}


class GpuExecutor:
    """The library on the GPU: a domain per request, batches of domains."""

    def footprint(self, req):
        return footprint(req)

    def create(self, req):
        return B.build_domain(req)

    def run_alone(self, dom, steps):
        dom.step(int(steps))
        dom.sync()

    def result(self, dom):
        return _result(dom)

    def destroy(self, dom):
        dom.close()

    def new_batch(self, use_graph=True, launch=None):
        bt = B.Batch()
        if use_graph:
            bt.set("use_graph", 1)
        if launch:
            bt.set("block", launch[0])
            bt.set("step_flags", launch[1])
        return bt

    def batch_add(self, bt, dom):
        bt.add(dom)

    def batch_remove(self, bt, dom):
        bt.remove(dom)

    def batch_step(self, bt, n):
        bt.step(int(n))
        bt.sync()

    def batch_close(self, bt):
        bt.close()


class ContinuousServer:
    """Continuous batching with admission by HBM footprint."""

    def __init__(self, budget_bytes, max_slots=64, chunk=50, use_graph=True, keep_results=False, launch=None,
                 executor=None):
        self.ex = executor or GpuExecutor()
        self.budget = budget_bytes
        self.max_slots = max_slots
        self.chunk = chunk
        self.batch = self.ex.new_batch(use_graph, launch)
        self.active = {}  # rid -> [domain, request, arrival, remaining, footprint]
        self.used = 0
        self.keep = keep_results
        self.peak_used = 0
        self.peak_slots = 0

    def can_admit(self, req):
        return len(self.active) < self.max_slots and self.used + self.ex.footprint(req) <= self.budget

    def admit(self, rid, req, arrival):
        d = self.ex.create(req)
        fp = self.ex.footprint(req)
        self.ex.batch_add(self.batch, d)
        self.active[rid] = [d, req, arrival, int(req["steps"]), fp]
        self.used += fp
        self.peak_used = max(self.peak_used, self.used)
        self.peak_slots = max(self.peak_slots, len(self.active))

    def step(self):
        """Advance every active request by one chunk (never past its end)."""
        n = min(self.chunk, min(v[3] for v in self.active.values()))
        self.ex.batch_step(self.batch, n)
        for v in self.active.values():
            v[3] -= n
        return n

    def retire(self, stats, now):
        for rid in [r for r, v in self.active.items() if v[3] == 0]:
            d, req, arrival, _, fp = self.active.pop(rid)
            res = self.ex.result(d) if self.keep else None
            self.ex.batch_remove(self.batch, d)
            self.ex.destroy(d)
            self.used -= fp
            stats.done(rid, req, arrival, now, res)

    def close(self):
        for v in self.active.values():
            self.ex.batch_remove(self.batch, v[0])
            self.ex.destroy(v[0])
        self.active.clear()
        self.ex.batch_close(self.batch)


def run_continuous(trace, budget_bytes, max_slots=64, chunk=50, keep_results=False, launch=None, executor=None,
                   clock=None):
    clk = clock or WallClock()
    srv = ContinuousServer(budget_bytes, max_slots, chunk, keep_results=keep_results, launch=launch,
                           executor=executor)
    st = Stats()
    queue = []
    i = 0
    try:
        while i < len(trace) or queue or srv.active:
            now = clk.now()
            while i < len(trace) and trace[i][0] <= now:
                queue.append((i, trace[i][1], trace[i][0]))
                i += 1
            st.max_queue = max(st.max_queue, len(queue))
            while queue and srv.can_admit(queue[0][1]):
                rid, req, arr = queue.pop(0)
                st.trace_log.append(("admit", rid, clk.now()))
                srv.admit(rid, req, arr)
            if queue and not srv.active:
                raise RuntimeError("request %d does not fit the memory budget" % queue[0][0])
            if srv.active:
                srv.step()
                srv.retire(st, clk.now())
            elif i < len(trace):
                clk.sleep(max(0.0, min(trace[i][0] - now, 0.05)))
        wall = clk.now()
    finally:
        srv.close()
    st.peak_used, st.peak_slots = srv.peak_used, srv.peak_slots
    return st, wall


def run_fifo(trace, keep_results=False, executor=None, clock=None):
    ex = executor or GpuExecutor()
    clk = clock or WallClock()
    st = Stats()
    for rid, (arr, req) in enumerate(trace):
        now = clk.now()
        if now < arr:
            clk.sleep(arr - now)
        st.max_queue = max(st.max_queue, sum(1 for a, _ in trace[rid:] if a <= clk.now()))
        st.trace_log.append(("admit", rid, clk.now()))
        d = ex.create(req)
        try:
            ex.run_alone(d, req["steps"])
            res = ex.result(d) if keep_results else None
        finally:
            ex.destroy(d)
        st.done(rid, req, arr, clk.now(), res)
    return st, clk.now()


def run_static(trace, batch_size=16, max_wait=0.5, keep_results=False, executor=None, clock=None):
    """Wait for up to batch_size arrived requests (at most max_wait after the
    first), run them together to completion, repeat."""
    ex = executor or GpuExecutor()
    clk = clock or WallClock()
    st = Stats()
    i = 0
    while i < len(trace):
        now = clk.now()
        if trace[i][0] > now:
            clk.sleep(trace[i][0] - now)
        first = clk.now()
        while True:
            now = clk.now()
            ready = sum(1 for a, _ in trace[i:i + batch_size] if a <= now)
            if ready >= batch_size or now - first >= max_wait or i + ready >= len(trace):
                break
            clk.sleep(0.005)
        group = list(range(i, i + max(ready, 1)))
        i += len(group)
        st.max_queue = max(st.max_queue, len(group))
        bt = ex.new_batch(True)
        doms = []
        try:
            for rid in group:
                st.trace_log.append(("admit", rid, clk.now()))
                d = ex.create(trace[rid][1])
                ex.batch_add(bt, d)
                doms.append([rid, d, int(trace[rid][1]["steps"])])
            while doms:
                n = min(v[2] for v in doms)
                ex.batch_step(bt, n)
                now = clk.now()
                keep = []
                for v in doms:
                    v[2] -= n
                    if v[2] == 0:
                        res = ex.result(v[1]) if keep_results else None
                        ex.batch_remove(bt, v[1])
                        ex.destroy(v[1])
                        st.done(v[0], trace[v[0]][1], trace[v[0]][0], now, res)
                    else:
                        keep.append(v)
                doms = keep
        finally:
            for v in doms:
                ex.batch_remove(bt, v[1])
                ex.destroy(v[1])
            ex.batch_close(bt)
    return st, clk.now()


def default_budget():
    try:
        import torch
        free, total = torch.cuda.mem_get_info()
        return int(0.6 * free)
    except Exception:
        return 64 << 30


DISABLED = ("the serving benchmark at production scale (Poisson 20 req/s, 32^3-128^3 requests, chunk 50) ended "
            "in a host segmentation fault on the GPU without a diagnosed cause; it stays off the GPU until one is "
            "found (the request loop is covered by the served-equals-alone and served-vs-oracle GPU tests and by "
            "the virtual-clock tests of its logic)")


def bench(args):
    """Replay a Poisson trace (rate 20/s) in the three modes."""
    if not getattr(args, "force", False):
        raise RuntimeError(DISABLED)
    rate = getattr(args, "rate", None) or 20.0
    duration = getattr(args, "duration", None) or 15.0
    trace = W.serving_trace(rate=rate, duration=duration, seed=5)
    out = {"metric": "served vs plain (Poisson request stream)", "rate_per_s": rate, "duration_s": duration,
           "requests": len(trace),
           "offered_MLUPS": sum(nodes_of(r) * r["steps"] for _, r in trace) / duration / 1e6}
    budget = default_budget()
    st, wall = run_continuous(trace, budget)
    out["continuous"] = st.summary(wall)
    st, wall = run_static(trace)
    out["static"] = st.summary(wall)
    st, wall = run_fifo(trace)
    out["fifo"] = st.summary(wall)
    out["budget_bytes"] = budget
    print(json.dumps(out), flush=True)
