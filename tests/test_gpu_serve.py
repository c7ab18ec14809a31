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
    # the per-bulk timings: issued after the cut and before the results were
    # back; the device times are measured, non-negative and no longer than
    # the bulk's time from issue to completion
    assert np.all(recs["issued_ns"] >= recs["cut_ns"])
    assert np.all(recs["done_ns"] >= recs["issued_ns"])
    assert np.all(recs["front_us"] >= 0) and np.all(recs["exec_us"] >= 0)
    assert np.all(recs["exec_us"] * 1000 <= recs["done_ns"] - recs["cut_ns"] + 1000)
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


def test_live_server_submit_poll_matches_oracle():
    """gputx_serve_open/submit/poll/close: signatures submitted in uneven
    pieces while earlier bulks run, results polled as they finish.  Every
    ticket's status and results, and the tables read back through
    gputx_read_table, equal the oracle run over all submissions in order."""
    import time
    import torch
    from paper_1103_3105_amd import gputx
    rng = np.random.default_rng(34)
    tabs = wl.sub_tables(rng, 10_000, occupancy=0.4)
    bulk = wl.sub_bulk(rng, 30_000, 10_000, 0.8)
    eng = gputx.Engine(tabs, wl.sub_types(), part_size=16)
    got_t, got_s, got_r, got_l = [], [], [], []
    try:
        srv = serving.Server(eng, bulk.params.shape[0], 14, deadline_us=150, slots=3, max_bulk=4096,
                             pool_capacity=40_000)
        try:
            pos, sizes = 0, [1, 7, 500, 3000, 64, 9000, 2500, 15000]
            for k, m in enumerate(sizes):
                m = min(m, bulk.n - pos)
                first = srv.submit(bulk.type[pos:pos + m], bulk.params[:, pos:pos + m], bulk.ts[pos:pos + m])
                assert first == pos
                pos += m
                time.sleep(0.0002 * (k % 3))
                t, s, r, l = srv.poll()
                got_t.append(t); got_s.append(s); got_r.append(r); got_l.append(l)
            if pos < bulk.n:
                srv.submit(bulk.type[pos:], bulk.params[:, pos:], bulk.ts[pos:])
            deadline = time.time() + 30
            while sum(len(x) for x in got_t) < bulk.n and time.time() < deadline:
                t, s, r, l = srv.poll()
                got_t.append(t); got_s.append(s); got_r.append(r); got_l.append(l)
        finally:
            rep = srv.close()
        torch.cuda.synchronize()
        g_sub = [gputx.gputx_read_table(eng.h, eng.table_id["subscriber"], c, 0, 10_000,
                                        np.int64 if c == 0 else np.int32) for c in range(15)]
        g_cf = [gputx.gputx_read_table(eng.h, eng.table_id["call_fwd"], c, 0, 120_000,
                                       np.int64 if c == 2 else np.int32) for c in range(3)]
    finally:
        eng.close()
    tk = np.concatenate(got_t)
    assert np.array_equal(tk, np.arange(bulk.n))         # every ticket once, in order
    o_tabs = util.copy_tables(tabs)
    rc, o_st, o_res = oracle.run_serial(o_tabs, wl.sub_types(), bulk.type, bulk.params, bulk.ts, 14)
    assert rc == 0
    assert np.array_equal(np.concatenate(got_s), o_st)
    assert np.array_equal(np.concatenate(got_r), o_res)
    assert np.all(np.concatenate(got_l) > 0)
    for c in range(15):
        assert np.array_equal(g_sub[c], o_tabs["subscriber"].cols[c]), c
    for c in range(3):
        assert np.array_equal(g_cf[c], o_tabs["call_fwd"].cols[c]), c
    assert rep.committed == int((o_st == 0).sum()) and rep.n_bulks >= 2


def test_live_server_pool_capacity_and_order():
    """A full pool refuses a submission (nothing taken) until results are
    polled; ids that do not ascend are refused."""
    import time
    from paper_1103_3105_amd import gputx
    rng = np.random.default_rng(35)
    tabs = wl.sub_tables(rng, 2000, occupancy=0.4)
    bulk = wl.sub_bulk(rng, 1500, 2000, 0.8)
    eng = gputx.Engine(tabs, wl.sub_types(), part_size=16)
    try:
        srv = serving.Server(eng, bulk.params.shape[0], 14, deadline_us=100, slots=2, max_bulk=1024,
                             pool_capacity=1000)
        try:
            srv.submit(bulk.type[:800], bulk.params[:, :800], bulk.ts[:800])
            with pytest.raises(gputx.GputxError) as ei:
                srv.submit(bulk.type[800:1100], bulk.params[:, 800:1100], bulk.ts[800:1100])
            assert ei.value.code == gputx.E_CAPACITY
            with pytest.raises(gputx.GputxError) as ei:   # id below the last one
                srv.submit(bulk.type[:5], bulk.params[:, :5], bulk.ts[:5])
            assert ei.value.code == gputx.E_ARG
            n_got, deadline = 0, time.time() + 30
            while n_got < 800 and time.time() < deadline:
                n_got += len(srv.poll()[0])
            assert n_got == 800
            assert srv.submit(bulk.type[800:1100], bulk.params[:, 800:1100], bulk.ts[800:1100]) == 800
        finally:
            srv.close()
    finally:
        eng.close()


def test_read_table_bounds():
    from paper_1103_3105_amd import gputx
    rng = np.random.default_rng(36)
    tabs = wl.sub_tables(rng, 3000, occupancy=0.4)
    eng = gputx.Engine(tabs, wl.sub_types(), part_size=16)
    try:
        tid = eng.table_id["subscriber"]
        got = gputx.gputx_read_table(eng.h, tid, 3, 1000, 500, np.int32)
        assert np.array_equal(got, tabs["subscriber"].cols[3][1000:1500])
        for bad in ((tid, 3, 2900, 200), (tid, 99, 0, 1), (31, 0, 0, 1), (tid, 0, -1, 2)):
            with pytest.raises(gputx.GputxError) as ei:
                gputx.gputx_read_table(eng.h, *bad, np.int64)
            assert ei.value.code == gputx.E_ARG
    finally:
        eng.close()
