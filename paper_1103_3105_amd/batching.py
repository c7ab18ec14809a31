"""Batched form: many uneven bulks over two databases in one graph launch.

The bank and the order-entry databases live in one context; every bulk
belongs to one of them (a *lane*).  Bulks of one lane run in submission
order, the two lanes run concurrently, and within a lane the bulk generation
of the next bulk overlaps the execution of the current one (``gputx_batch_*``
in the C ABI).  The plain form runs the same bulks one ``gputx_execute_bulk``
at a time, waiting for each bulk's results before the next (a client that
needs its results).
"""
from __future__ import annotations

import dataclasses
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import workloads as wl

LANE = {"bank": 0, "order": 1}
WIDTH = {"bank": 3, "order": 16}
MAX_OPS = {"bank": 3, "order": 15}


@dataclasses.dataclass
class BatchWorkload:
    tables: Dict[str, wl.Table]       # both databases
    types: List[wl.TypeDesc]
    jobs: List[tuple]                 # (db, Bulk) in submission order
    name: str

    @property
    def n_txns(self) -> int:
        return sum(b.n for _, b in self.jobs)


def config4(n_bulks: int = 512, lo: int = 256, hi: int = 262_144, repeats: int = 1,
            bank_branches: int = 64, accounts_per_branch: int = 100_000, n_wh: int = 16,
            items_per_w: int = 100_000, c_per_d: int = 3000) -> BatchWorkload:
    """512 bulks, log-uniform sizes in [lo, hi], each a bank bulk (Zipf theta
    drawn from {0, 0.8, 0.99}) or an order-entry bulk by coin flip.  Append
    tables are sized for ``repeats`` executions of the whole batch."""
    bank, order, seq = wl.config4(n_bulks, lo, hi, bank_branches=bank_branches,
                                  accounts_per_branch=accounts_per_branch, n_wh=n_wh,
                                  items_per_w=items_per_w, c_per_d=c_per_d)
    tables = {}
    for src in (bank, order):
        for name, t in src.tables.items():
            if t.append and repeats > 1:
                cap = t.capacity * repeats
                t = wl.Table(t.name, t.dtypes, [np.zeros(cap, c.dtype) for c in t.cols], 0, cap,
                             append=True)
            tables[name] = t
    jobs = [(db, (bank if db == "bank" else order).bulks[k]) for db, k in seq]
    return BatchWorkload(tables, bank.types + order.types, jobs,
                         f"batch-{n_bulks}x[{lo},{hi}]")


def sequence(bw: BatchWorkload):
    """(bulk, result width) of every job in submission order."""
    return [(b, WIDTH[db]) for db, b in bw.jobs]


def device_jobs(eng, bw: BatchWorkload, strategy: int) -> List[dict]:
    jobs = []
    for db, b in bw.jobs:
        jobs.append(dict(dev=eng.bulk_to_device(b), lane=LANE[db], strategy=strategy,
                         width=WIDTH[db], ts_sorted=True, max_ops=MAX_OPS[db], db=db))
    return jobs


def run_plain(eng, jobs: Sequence[dict], outputs: Optional[list] = None):
    """One gputx_execute_bulk per bulk on one stream, waiting for each."""
    import torch
    stream = torch.cuda.current_stream()
    lat = []
    for k, j in enumerate(jobs):
        o = outputs[k] if outputs else {}
        t0 = time.perf_counter()
        eng.execute(j["dev"], j["strategy"], j["width"], ts_sorted=True,
                    status=o.get("status"), results=o.get("results"), stats=o.get("stats"),
                    stream=stream)
        stream.synchronize()
        lat.append(time.perf_counter() - t0)
    return np.array(lat)
