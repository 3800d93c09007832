"""Serving: a request loop over a Poisson stream of independent solves.

Continuous batching (`ContinuousServer`): every request is a domain whose
state stays in HBM from admission to completion.  At each chunk boundary the
server admits queued requests in arrival order while their device footprint
(rwmi_footprint_bytes) fits the memory budget and a slot is free, steps all
admitted domains together (one rwmi batch: every kernel of a step is one
launch over all members), and retires the ones that reached their step count
(reads their moments, frees their memory).  Requests that arrive while others
run therefore start as soon as memory and a slot free up, and their work
overlaps on the device.

Baselines on the same trace: `fifo` runs each request alone, one after the
other; `static` waits for a batch of requests, runs the batch to completion
without admitting newcomers, then forms the next.

Latency is measured from arrival to completion (wall clock, seconds since
the start of the trace replay).  A request's result does not depend on what
else is in the batch (same arithmetic per node and per walker).
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


class Stats:
    def __init__(self):
        self.lat = []
        self.node_steps = 0
        self.walker_steps = 0
        self.max_queue = 0
        self.results = {}

    def done(self, rid, req, arrival, now, result=None):
        self.lat.append(now - arrival)
        self.node_steps += nodes_of(req) * req["steps"]
        self.walker_steps += req["walkers"]["n"] * req["steps"]
        if result is not None:
            self.results[rid] = result

    def summary(self, wall):
        lat = np.array(self.lat) if self.lat else np.array([np.nan])
        return {"completed": len(self.lat), "p50_s": float(np.percentile(lat, 50)),
                "p99_s": float(np.percentile(lat, 99)), "mean_s": float(np.mean(lat)), "wall_s": wall,
                "MLUPS": self.node_steps / wall / 1e6, "walker_steps_per_s": self.walker_steps / wall,
                "max_queue": self.max_queue}


def _result(d):
    m = d.moments()
    return {"step": m["step"], "n_walkers": m["n_walkers"], "sum": m["sum"].tolist(), "sumsq": m["sumsq"].tolist(),
            "mass": m["mass"], "counters": m["counters"]}


class ContinuousServer:
    """Continuous batching with admission by HBM footprint."""

    def __init__(self, budget_bytes, max_slots=64, chunk=50, use_graph=True, keep_results=False, launch=None):
        self.budget = budget_bytes
        self.max_slots = max_slots
        self.chunk = chunk
        self.batch = B.Batch()
        if use_graph:
            self.batch.set("use_graph", 1)
        if launch:
            self.batch.set("block", launch[0])
            self.batch.set("step_flags", launch[1])
        self.active = {}  # rid -> [domain, request, arrival, remaining, footprint]
        self.used = 0
        self.keep = keep_results

    def can_admit(self, req):
        return len(self.active) < self.max_slots and self.used + footprint(req) <= self.budget

    def admit(self, rid, req, arrival):
        d = B.build_domain(req)
        fp = footprint(req)
        self.batch.add(d)
        self.active[rid] = [d, req, arrival, int(req["steps"]), fp]
        self.used += fp

    def step(self):
        """Advance every active request by one chunk (never past its end)."""
        n = min(self.chunk, min(v[3] for v in self.active.values()))
        self.batch.step(n)
        self.batch.sync()
        for v in self.active.values():
            v[3] -= n
        return n

    def retire(self, stats, now):
        for rid in [r for r, v in self.active.items() if v[3] == 0]:
            d, req, arrival, _, fp = self.active.pop(rid)
            res = _result(d) if self.keep else None
            self.batch.remove(d)
            d.close()
            self.used -= fp
            stats.done(rid, req, arrival, now, res)

    def close(self):
        for v in self.active.values():
            self.batch.remove(v[0])
            v[0].close()
        self.active.clear()
        self.batch.close()


def run_continuous(trace, budget_bytes, max_slots=64, chunk=50, keep_results=False, launch=None):
    srv = ContinuousServer(budget_bytes, max_slots, chunk, keep_results=keep_results, launch=launch)
    st = Stats()
    queue = []
    i = 0
    t0 = time.perf_counter()
    while i < len(trace) or queue or srv.active:
        now = time.perf_counter() - t0
        while i < len(trace) and trace[i][0] <= now:
            queue.append((i, trace[i][1], trace[i][0]))
            i += 1
        st.max_queue = max(st.max_queue, len(queue))
        while queue and srv.can_admit(queue[0][1]):
            rid, req, arr = queue.pop(0)
            srv.admit(rid, req, arr)
        if queue and not srv.active:
            raise RuntimeError("request %d does not fit the memory budget" % queue[0][0])
        if srv.active:
            srv.step()
            srv.retire(st, time.perf_counter() - t0)
        elif i < len(trace):
            time.sleep(max(0.0, min(trace[i][0] - now, 0.05)))
    wall = time.perf_counter() - t0
    srv.close()
    return st, wall


def run_fifo(trace, keep_results=False):
    st = Stats()
    t0 = time.perf_counter()
    for rid, (arr, req) in enumerate(trace):
        now = time.perf_counter() - t0
        if now < arr:
            time.sleep(arr - now)
        st.max_queue = max(st.max_queue, sum(1 for a, _ in trace[rid:] if a <= time.perf_counter() - t0))
        d = B.build_domain(req)
        d.step(int(req["steps"]))
        d.sync()
        res = _result(d) if keep_results else None
        d.close()
        st.done(rid, req, arr, time.perf_counter() - t0, res)
    return st, time.perf_counter() - t0


def run_static(trace, batch_size=16, max_wait=0.5, keep_results=False):
    """Wait for up to batch_size arrived requests (at most max_wait after the
    first), run them together to completion, repeat."""
    st = Stats()
    t0 = time.perf_counter()
    i = 0
    while i < len(trace):
        now = time.perf_counter() - t0
        if trace[i][0] > now:
            time.sleep(trace[i][0] - now)
        first = time.perf_counter() - t0
        while True:
            now = time.perf_counter() - t0
            ready = sum(1 for a, _ in trace[i:i + batch_size] if a <= now)
            if ready >= batch_size or now - first >= max_wait or i + ready >= len(trace):
                break
            time.sleep(0.005)
        group = list(range(i, i + max(ready, 1)))
        i += len(group)
        st.max_queue = max(st.max_queue, len(group))
        bt = B.Batch()
        bt.set("use_graph", 1)
        doms = []
        for rid in group:
            d = B.build_domain(trace[rid][1])
            bt.add(d)
            doms.append([rid, d, int(trace[rid][1]["steps"])])
        while doms:
            n = min(v[2] for v in doms)
            bt.step(n)
            bt.sync()
            now = time.perf_counter() - t0
            keep = []
            for v in doms:
                v[2] -= n
                if v[2] == 0:
                    res = _result(v[1]) if keep_results else None
                    bt.remove(v[1])
                    v[1].close()
                    st.done(v[0], trace[v[0]][1], trace[v[0]][0], now, res)
                else:
                    keep.append(v)
            doms = keep
        bt.close()
    return st, time.perf_counter() - t0


def default_budget():
    try:
        import torch
        free, total = torch.cuda.mem_get_info()
        return int(0.6 * free)
    except Exception:
        return 64 << 30


DISABLED = ("the serving benchmark at production scale (Poisson 20 req/s, 32^3-128^3 requests, chunk 50) ended "
            "in a host segmentation fault on the GPU without a diagnosed cause; it stays disabled until one is found "
            "(the request loop itself is covered by the small served-equals-alone tests)")


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
