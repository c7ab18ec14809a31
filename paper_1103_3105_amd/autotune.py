"""Calibration of Algorithm 1 and of the executors' launch shapes.

Appendix D leaves the thresholds of Algorithm 1 (w0_bar, c_bar, d_bar) to
calibration.  ``calibrate`` runs sample bulks under every strategy on a
scratch copy of the database (so the real tables are untouched), records the
bulk's features (w0, depth, cross-partition count c) and each strategy's
time, and picks the thresholds that minimise the total time Algorithm 1
would have spent on the samples.  It also picks K-SET's narrow-wave width
and the persistent grid size from a small candidate set.

``tune_buckets`` tunes per bulk shape instead (database and size class): for
each bucket it times a sample bulk under every executor and a set of launch
shapes (persistent grid, K-SET narrow-wave width) and keeps the fastest; the
batched form then runs every bulk with its bucket's choice.
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import Dict, List, Sequence

import numpy as np

STRATS = ("TPL", "PART", "KSET")


@dataclasses.dataclass
class Sample:
    w0: int
    depth: int
    cross: int
    ms: Dict[str, float]      # strategy -> ms


def choose(w0, depth, cross, w0_bar, c_bar, d_bar) -> str:
    """Algorithm 1 (Appendix D)."""
    if w0 >= w0_bar:
        return "KSET"
    if cross <= c_bar or depth >= d_bar:
        return "PART" if cross == 0 else "TPL"  # PART with c > 0 runs under TPL (Section 5.2)
    return "TPL"


def fit_thresholds(samples: Sequence[Sample]):
    """Grid search over thresholds taken from the samples' own feature values.
    c_bar = -1 lets Algorithm 1 reach TPL for shallow bulks without
    cross-partition transactions (PART then needs depth >= d_bar)."""
    big = 1 << 40
    w0s = sorted({s.w0 for s in samples} | {big})
    ds = sorted({s.depth for s in samples} | {0, big})
    cs = sorted({-1, 0} | {s.cross for s in samples})
    best = None
    for w0_bar, c_bar, d_bar in itertools.product(w0s, cs, ds):
        tot = sum(s.ms[choose(s.w0, s.depth, s.cross, w0_bar, c_bar, d_bar)] for s in samples)
        if best is None or tot < best[0] - 1e-9:
            best = (tot, w0_bar, c_bar, d_bar)
    return {"w0_bar": best[1], "c_bar": best[2], "d_bar": best[3], "total_ms": best[0]}


def _time(eng, dev, strategy, width, max_ops, reps=2):
    import torch
    from . import gputx
    stream = torch.cuda.current_stream()
    eng.truncate_appends()
    outs = eng.execute(dev, gputx.STRATEGY[strategy], width, ts_sorted=True, stream=stream)  # warm
    tot = 0.0
    for _ in range(reps):
        eng.truncate_appends()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        eng.execute(dev, gputx.STRATEGY[strategy], width, ts_sorted=True, status=outs[0],
                    results=outs[1], stats=outs[2], stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        tot += a.elapsed_time(b)
    return tot / reps, gputx.stats_from(outs[2])


def calibrate(tables, types, sample_bulks: Sequence[tuple], narrow=(64, 256, 1024),
              grids=(0,), log=None, engine_opts=None) -> dict:
    """sample_bulks: (Bulk, width, max_ops) tuples.  Returns the options to set
    (w0_bar, c_bar, d_bar, kset_narrow, grid_blocks) and the samples.
    engine_opts: options of the engine the thresholds are for (part_size ...)."""
    from . import gputx
    scratch = {k: v.copy() for k, v in tables.items()}
    for t in scratch.values():   # room for one sample run's appends (emptied between runs)
        if t.append:
            cap = max(b.n for b, _, _ in sample_bulks) * 16
            t.cols = [np.zeros(cap, c.dtype) for c in t.cols]
            t.capacity, t.n_rows = cap, 0
    eng = gputx.Engine(scratch, types, **(engine_opts or {}))
    samples: List[Sample] = []
    try:
        best_narrow, best_grid = None, None
        # launch shapes first, on the samples K-SET runs (narrow width) and TPL runs (grid)
        shape_ms = {}
        for nw, gb in itertools.product(narrow, grids):
            eng.set_options(kset_narrow=nw, grid_blocks=gb)
            tot = 0.0
            for b, width, mo in sample_bulks:
                dev = eng.bulk_to_device(b)
                tot += _time(eng, dev, "KSET", width, mo, reps=1)[0]
            shape_ms[(nw, gb)] = tot
        best_narrow, best_grid = min(shape_ms, key=shape_ms.get)
        eng.set_options(kset_narrow=best_narrow, grid_blocks=best_grid)
        for b, width, mo in sample_bulks:
            dev = eng.bulk_to_device(b)
            ms, feats = {}, None
            for strat in STRATS:
                ms[strat], st = _time(eng, dev, strat, width, mo)
                feats = feats or st
            samples.append(Sample(int(feats.w0), int(feats.depth), int(feats.cross), ms))
            if log:
                log(f"[tune] n={b.n} w0={feats.w0} d={feats.depth} c={feats.cross} " +
                    " ".join(f"{k}={v:.2f}" for k, v in ms.items()))
    finally:
        eng.close()
    th = fit_thresholds(samples)
    th.update(kset_narrow=best_narrow, grid_blocks=best_grid,
              samples=[dataclasses.asdict(s) for s in samples])
    return th


def tune_part_size(tables, types, sample_bulks: Sequence[tuple], sizes=(1, 4, 16, 64, 256, 1024),
                   log=None, engine_opts=None) -> dict:
    """Section 5.2's tuning parameter: the partition size (root keys per
    partition) PART runs fastest with on the sample bulks, from a candidate
    set (Appendix F.1 measures PART across partition sizes).  Each candidate
    runs every sample under PART on a scratch copy of the database; a bulk
    whose transactions cross partitions at that size runs under TPL (Section
    5.2), and its time counts as it is.  Returns {best, ms: {size: total ms},
    ran: {size: executors that ran}}."""
    from . import gputx
    scratch = {k: v.copy() for k, v in tables.items()}
    for t in scratch.values():
        if t.append:
            cap = max(b.n for b, _, _ in sample_bulks) * 16
            t.cols = [np.zeros(cap, c.dtype) for c in t.cols]
            t.capacity, t.n_rows = cap, 0
    eng = gputx.Engine(scratch, types, **(engine_opts or {}))
    ms, ran = {}, {}
    try:
        for size in sizes:
            eng.set_options(part_size=int(size))
            tot, labels = 0.0, set()
            for b, width, mo in sample_bulks:
                dev = eng.bulk_to_device(b)
                t, st = _time(eng, dev, "PART", width, mo, reps=1)
                tot += t
                labels.add(st.label)
            ms[int(size)] = round(tot, 4)
            ran[int(size)] = sorted(labels)
            if log:
                log(f"[tune] part_size={size}: {tot:.3f} ms ({', '.join(sorted(labels))})")
    finally:
        eng.close()
    return dict(best=min(ms, key=ms.get), ms=ms, ran=ran)


def bucket_of(db: str, n: int) -> tuple:
    """Shape bucket of a bulk: its database and the power of two below its size."""
    return (db, max(0, int(n).bit_length() - 1))


def tune_buckets(tables, types, jobs: Sequence[tuple], width: Dict[str, int], max_ops: Dict[str, int],
                 grids=(64, 128, 256, 512), narrow=(64, 256, 1024), log=None, engine_opts=None) -> dict:
    """Per shape bucket (database, log2 of the bulk size), the executor and
    launch shape that ran a sample bulk of the bucket fastest on a scratch
    copy of the database: strategy (TPL, PART or K-SET), the persistent grid
    of TPL and K-SET, and K-SET's narrow-wave width.

    jobs: (db, Bulk) pairs; the sample of a bucket is its median-size bulk.
    A launch shape is tried only for an executor that came within twice the
    best time so far with the default shape.  Returns {bucket: {strategy,
    grid_blocks, kset_narrow, ms, tried}}."""
    from . import gputx
    by_bucket: Dict[tuple, list] = {}
    for db, b in jobs:
        by_bucket.setdefault(bucket_of(db, b.n), []).append((db, b))
    scratch = {k: v.copy() for k, v in tables.items()}
    biggest = max(b.n for _, b in jobs)
    for t in scratch.values():
        if t.append:
            cap = biggest * 16
            t.cols = [np.zeros(cap, c.dtype) for c in t.cols]
            t.capacity, t.n_rows = cap, 0
    eng = gputx.Engine(scratch, types, **(engine_opts or {}))
    out = {}
    try:
        for key in sorted(by_bucket):
            group = sorted(by_bucket[key], key=lambda j: j[1].n)
            db, b = group[len(group) // 2]
            dev = eng.bulk_to_device(b)
            tried = {}

            def run(strat, gb, nw):
                eng.set_options(grid_blocks=gb, kset_narrow=nw)
                ms, _ = _time(eng, dev, strat, width[db], max_ops[db], reps=1)
                tried[f"{strat}/{gb}/{nw}"] = round(ms, 4)
                return ms

            best = ("PART", 0, 256, run("PART", 0, 256))
            for strat in ("TPL", "KSET"):
                ms = run(strat, 0, 256)
                if ms < best[3]:
                    best = (strat, 0, 256, ms)
                if ms > 2 * best[3]:
                    continue
                for gb in grids:
                    for nw in (narrow if strat == "KSET" else (256,)):
                        if (gb, nw) == (0, 256):
                            continue
                        m2 = run(strat, gb, nw)
                        if m2 < best[3]:
                            best = (strat, gb, nw, m2)
            out[key] = dict(strategy=best[0], grid_blocks=best[1], kset_narrow=best[2],
                            ms=round(best[3], 4), tried=tried, sample_n=b.n)
            if log:
                log(f"[tune] bucket {key}: {best[0]} grid={best[1]} narrow={best[2]} "
                    f"{best[3]:.3f} ms (sample n={b.n}, {len(tried)} runs)")
    finally:
        eng.close()
    return out
