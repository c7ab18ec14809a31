"""Served form: a live server (``gputx_serve_open`` / submit / poll / close)
and a Poisson arrival trace replayed through it (``gputx_serve``).

Arrivals follow a Poisson process of rate lambda; each arrival is a
subscriber transaction (mix and key skew of the subscriber workload).  The
native serving loop cuts a bulk every deadline, keeps up to ``slots`` bulks in
flight and returns per-bulk completion times, from which every transaction's
commit latency (result back in host memory minus arrival) follows.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import workloads as wl


@dataclasses.dataclass
class Trace:
    arrival_ns: np.ndarray   # int64 [n], non-decreasing
    type: np.ndarray         # int32 [n]
    params: np.ndarray       # int64 [P, n]
    ts: np.ndarray           # int64 [n] ascending

    @property
    def n(self) -> int:
        return int(self.type.shape[0])


def make_trace(rate_per_s: float, duration_s: float, n_sub: int, theta: float = 0.8,
               seed: int = 0) -> Trace:
    """Poisson arrivals at ``rate_per_s`` for ``duration_s`` seconds; transaction
    ids (timestamps) follow arrival order."""
    rng = wl.rng_for(5, 10 + seed)
    arr = wl.poisson_arrivals(rng, rate_per_s, duration_s)
    bulk = wl.sub_bulk(rng, int(arr.shape[0]), n_sub, theta)
    return Trace(arr, bulk.type, bulk.params, np.arange(arr.shape[0], dtype=np.int64))


@dataclasses.dataclass
class ServeResult:
    status: np.ndarray
    results: np.ndarray
    bulks: np.ndarray          # per-bulk records (first, count, cut_ns, done_ns, error, slot)
    committed: int
    aborted: int
    invalid: int
    elapsed_ns: int
    slots_used: int
    slot_bytes: int
    latency_ns: np.ndarray     # per transaction

    def percentiles(self):
        lat = self.latency_ns
        return {"p50_us": float(np.percentile(lat, 50)) / 1e3,
                "p99_us": float(np.percentile(lat, 99)) / 1e3,
                "mean_us": float(lat.mean()) / 1e3}

    @property
    def throughput(self) -> float:
        return self.committed / (self.elapsed_ns / 1e9) if self.elapsed_ns else 0.0


def serve(eng, trace: Trace, deadline_us: float, slots: int = 4, width: int = 14,
          strategy: int = 0, max_bulk: int = 1 << 17, hbm_budget: int = 0,
          max_ops: int = 1) -> ServeResult:
    """Run ``gputx_serve`` over the trace on engine ``eng``."""
    import ctypes
    import torch
    from . import gputx
    n = trace.n
    arrival = np.ascontiguousarray(trace.arrival_ns, dtype=np.int64)
    typ = np.ascontiguousarray(trace.type, dtype=np.int32)
    params = np.ascontiguousarray(trace.params, dtype=np.int64)
    ts = np.ascontiguousarray(trace.ts, dtype=np.int64)
    tr = gputx.Trace()
    tr.n = n
    tr.arrival_ns = arrival.ctypes.data
    tr.type = typ.ctypes.data
    tr.params = params.ctypes.data
    tr.n_params = params.shape[0]
    tr.ts = ts.ctypes.data
    o = gputx.ServeOpts()
    o.deadline_ns = int(deadline_us * 1000)
    o.slots = slots
    o.strategy = strategy
    o.max_bulk = max_bulk
    o.hbm_budget = hbm_budget
    o.width = width
    o.max_ops = max_ops
    status = torch.empty(max(n, 1), dtype=torch.int32).pin_memory()
    results = torch.empty((max(n, 1), width), dtype=torch.int64).pin_memory()
    dur = (arrival[-1] if n else 0) / 1e9
    cap = int(dur * 1e9 / o.deadline_ns) + n // max_bulk + 64
    rep, recs = gputx.gputx_serve(eng.h, tr, o, status, results, cap)
    st = status.numpy()[:n].copy()
    res = results.numpy()[:n].copy()
    lat = np.zeros(n, dtype=np.int64)
    for r in recs:
        f, c = int(r["first"]), int(r["count"])
        lat[f:f + c] = int(r["done_ns"]) - arrival[f:f + c]
    return ServeResult(st, res, recs, rep.committed, rep.aborted, rep.invalid, rep.elapsed_ns,
                       rep.slots_used, rep.slot_bytes, lat)


class Server:
    """A live server (``gputx_serve_open``): submit signatures as they
    arrive, poll finished transactions in submission order, close when done.

    Tickets are consecutive submission numbers starting at 0."""

    def __init__(self, eng, n_params: int, width: int, deadline_us: float, slots: int = 4,
                 strategy: int = 0, max_bulk: int = 1 << 17, hbm_budget: int = 0, max_ops: int = 1,
                 pool_capacity: int = 1 << 20):
        from . import gputx
        self._g = gputx
        self.eng = eng
        self.width = width
        o = gputx.ServeOpts()
        o.deadline_ns = int(deadline_us * 1000)
        o.slots = slots
        o.strategy = strategy
        o.max_bulk = max_bulk
        o.hbm_budget = hbm_budget
        o.width = width
        o.max_ops = max_ops
        self.s = gputx.gputx_serve_open(eng.h, o, n_params, pool_capacity)

    def submit(self, type_arr, params, ts) -> int:
        return self._g.gputx_serve_submit(self.eng.h, self.s, type_arr, params, ts)

    def poll(self, max_n: int = 1 << 16):
        return self._g.gputx_serve_poll(self.eng.h, self.s, max_n, self.width)

    def close(self):
        if self.s:
            s, self.s = self.s, None
            return self._g.gputx_serve_close(self.eng.h, s)
        return None
