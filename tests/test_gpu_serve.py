"""Served form (continuous batching over a Poisson trace) against the oracle.

Every transaction's status and results, and the final tables, must equal the
serial oracle run over the whole trace in arrival order -- whatever the bulk
boundaries and however many bulks overlapped on the device.  The per-bulk
records must partition the trace in order, each bulk holding only
transactions that had arrived when it was cut."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_1103_3105_amd import serving, workloads as wl
from tests import util

pytestmark = pytest.mark.gpu


def _check_records(res, trace, deadline_ns, max_bulk):
    recs = res.bulks
    assert recs.shape[0] >= 1
    first = recs["first"]
    count = recs["count"]
    assert first[0] == 0 and np.all(first[1:] == first[:-1] + count[:-1])
    assert first[-1] + count[-1] == trace.n
    assert np.all(count >= 1) and np.all(count <= max_bulk)
    assert np.all(recs["error"] == 0)
    last = first + count - 1
    # a bulk only holds transactions that had arrived by its cut
    assert np.all(trace.arrival_ns[last] <= recs["cut_ns"])
    assert np.all(recs["done_ns"] >= recs["cut_ns"])
    assert np.all(np.diff(recs["done_ns"]) >= 0)          # answered in issue order
    assert np.all(res.latency_ns > 0)


@pytest.mark.parametrize("deadline_us,slots,strategy", [(100, 4, 0), (1000, 2, 0), (300, 3, 3),
                                                        (300, 1, 1), (200, 4, 2)])
def test_served_equals_serial(deadline_us, slots, strategy):
    import torch
    from paper_1103_3105_amd import gputx
    rng = np.random.default_rng(31)
    tabs = wl.sub_tables(rng, 20_000, occupancy=0.4)
    trace = serving.make_trace(300_000, 0.25, 20_000, theta=0.8, seed=strategy)
    print("serve", deadline_us, slots, strategy, trace.n, file=sys.stderr, flush=True)
    eng = gputx.Engine(tabs, wl.sub_types(), part_size=16)
    try:
        res = serving.serve(eng, trace, deadline_us, slots=slots, width=14, strategy=strategy,
                            max_bulk=8192)
        torch.cuda.synchronize()
        g_tabs = util.copy_tables(tabs)
        for name, t in g_tabs.items():
            host = eng.table_host(name)
            for c in range(len(t.cols)):
                t.cols[c][:] = host[c]
    finally:
        eng.close()
    o_tabs = util.copy_tables(tabs)
    rc, o_st, o_res = oracle.run_serial(o_tabs, wl.sub_types(), trace.type, trace.params, trace.ts, 14)
    assert rc == 0
    assert np.array_equal(res.status, o_st)
    assert np.array_equal(res.results, o_res)
    ok, msg = util.tables_equal(o_tabs, g_tabs)
    assert ok, msg
    assert res.committed == int((o_st == 0).sum()) and res.aborted == int((o_st == 1).sum())
    assert res.invalid == 0
    _check_records(res, trace, deadline_us * 1000, 8192)


def test_hbm_budget_limits_slots():
    from paper_1103_3105_amd import gputx
    rng = np.random.default_rng(32)
    tabs = wl.sub_tables(rng, 5000, occupancy=0.4)
    trace = serving.make_trace(200_000, 0.05, 5000, seed=7)
    eng = gputx.Engine(tabs, wl.sub_types(), part_size=16)
    try:
        one = serving.serve(eng, trace, 200, slots=8, max_bulk=1024, hbm_budget=1)
    except gputx.GputxError as e:
        assert e.code == gputx.E_CAPACITY
    else:
        raise AssertionError("a budget below one slot must be refused")
    try:
        first = serving.serve(eng, trace, 200, slots=8, max_bulk=1024)
        assert first.slots_used == 8 and first.slot_bytes > 0
        res = serving.serve(eng, trace, 200, slots=8, max_bulk=1024,
                            hbm_budget=int(2.5 * first.slot_bytes))
        assert res.slots_used == 2
        _check_records(res, trace, 200_000, 1024)
    finally:
        eng.close()


def test_served_alone_equals_in_the_mix():
    """Continuous batching: with bulks overlapping on the device (4 slots)
    every transaction gets the same status and results, and the tables the
    same final state, as with bulks run one at a time (1 slot), whatever the
    bulk boundaries the two runs cut."""
    import torch
    from paper_1103_3105_amd import gputx
    rng = np.random.default_rng(33)
    tabs = wl.sub_tables(rng, 20_000, occupancy=0.4)
    trace = serving.make_trace(400_000, 0.1, 20_000, theta=0.8, seed=11)
    outs = []
    for slots in (1, 4):
        eng = gputx.Engine(util.copy_tables(tabs), wl.sub_types(), part_size=16)
        try:
            res = serving.serve(eng, trace, 100, slots=slots, width=14, max_bulk=4096)
            torch.cuda.synchronize()
            outs.append((res, {k: eng.table_host(k) for k in ("subscriber", "call_fwd")}))
        finally:
            eng.close()
    (r1, t1), (r4, t4) = outs
    assert r4.slots_used == 4 and r1.slots_used == 1
    assert np.array_equal(r1.status, r4.status)
    assert np.array_equal(r1.results, r4.results)
    for k in t1:
        assert all(np.array_equal(x, y) for x, y in zip(t1[k], t4[k])), k
