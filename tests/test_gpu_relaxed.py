"""Execution without the timestamp constraint (Appendix G) against the
oracle.

The relaxed executors only promise serializability: the result equals a
serial run in SOME order.  The engine reports that order as a key per
transaction (a logical clock of the locks under TPL, the grouped position
under PART).  The oracle then runs the bulk serially in key order; statuses,
results and every non-append table must agree exactly, and appended rows
must agree as a multiset (they take slots in input order on the GPU and in
serial order in the oracle)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_1103_3105_amd import workloads as wl
from tests import util

pytestmark = pytest.mark.gpu

TS_COL = {"history": 4, "orders": 0, "order_line": 0}


def run_relaxed(tabs, types, bulk, width, strategy, **opts):
    import torch
    from paper_1103_3105_amd import gputx
    eng = gputx.Engine(tabs, types, **opts)
    try:
        st, res, key, stats = eng.execute_relaxed(eng.bulk_to_device(bulk), gputx.STRATEGY[strategy], width)
        torch.cuda.synchronize()
        s = gputx.stats_from(stats)
        g_tabs = util.copy_tables(tabs)
        for name, t in g_tabs.items():
            host = eng.table_host(name)
            for c in range(len(t.cols)):
                t.cols[c][:] = host[c]
            if t.append:
                t.n_rows = eng.row_count(name)
        n = bulk.n
        return s, g_tabs, st.cpu().numpy()[:n], res.cpu().numpy()[:n], key.cpu().numpy()[:n]
    finally:
        eng.close()


def check_serializable(tabs, types, bulk, width, g_tabs, g_st, g_res, key):
    n = bulk.n
    assert np.array_equal(key < 0, g_st == oracle.INVALID)
    order = np.argsort(key, kind="stable")
    rank = np.empty(n, np.int64)
    rank[order] = np.arange(n)
    o_tabs = util.copy_tables(tabs)
    rc, o_st, o_res = oracle.run_serial(o_tabs, types, bulk.type, bulk.params, rank, width)
    assert rc == 0
    bad = np.flatnonzero(o_st != g_st)
    assert bad.size == 0, f"status differs at {bad[:8].tolist()}"
    bad = np.flatnonzero((o_res != g_res).any(axis=1))
    assert bad.size == 0, f"results differ at {bad[:8].tolist()}"
    for name, ot in o_tabs.items():
        gt = g_tabs[name]
        assert ot.n_rows == gt.n_rows, name
        if not ot.append:
            for c, (x, y) in enumerate(zip(ot.cols, gt.cols)):
                assert np.array_equal(x, y), (name, c)
            continue
        # the oracle wrote serial ranks as timestamps: map them back
        rows_o = np.stack([c[:ot.n_rows] for c in ot.cols], axis=1).copy()
        tc = TS_COL[name]
        rows_o[:, tc] = bulk.ts[order[rows_o[:, tc]]]
        rows_g = np.stack([c[:gt.n_rows] for c in gt.cols], axis=1)
        so = rows_o[np.lexsort(rows_o.T[::-1])]
        sg = rows_g[np.lexsort(rows_g.T[::-1])]
        assert np.array_equal(so, sg), name
    return o_st


@pytest.mark.parametrize("strategy", ["TPL", "PART"])
@pytest.mark.parametrize("workload", ["bank", "bank_remote", "order", "order_rb", "sub"])
def test_relaxed_is_serializable(workload, strategy):
    ps = 1
    if workload == "bank":
        tabs, types, bulk = util.small_bank(71, 20_000, n_branch=8, tpb=10, apt=300, theta=0.8)
        width = 3
    elif workload == "bank_remote":
        rng = np.random.default_rng(72)
        tabs = wl.bank_tables(rng, 8, 80, 24_000, history_capacity=20_000)
        bulk = wl.bank_bulk(rng, 20_000, 8, 80, 24_000, 0.8, remote_frac=0.05)
        types, width = wl.bank_types(), 3
    elif workload in ("order", "order_rb"):
        tabs, types, bulk = util.small_order(73, 20_000, n_wh=4, d_per_w=10, c_per_d=30, items_per_w=500,
                                             rollback_frac=0.05 if workload == "order_rb" else 0.0)
        width = 16
    else:
        tabs, types, bulk = util.small_sub(74, 20_000, n_sub=2000, theta=0.8)
        width, ps = 14, 16
    bulk = wl.shuffled(bulk, np.random.default_rng(9), gapped=True)   # input order is not ts order
    print("relaxed", workload, strategy, file=sys.stderr, flush=True)
    s, g_tabs, g_st, g_res, key = run_relaxed(tabs, types, bulk, width, strategy, part_size=ps)
    assert s.error == 0, s.as_dict()
    want = 2 if (strategy == "PART" and workload != "bank_remote") else 1
    assert s.chosen == want, s.as_dict()
    o_st = check_serializable(tabs, types, bulk, width, g_tabs, g_st, g_res, key)
    assert s.committed == int((o_st == 0).sum()) and s.aborted == int((o_st == 1).sum())
    if workload == "sub":
        assert s.aborted > 0


@pytest.mark.parametrize("strategy", ["TPL", "PART"])
@pytest.mark.parametrize("n", [0, 1, 2, 63, 4097])
def test_relaxed_small_bulks(n, strategy):
    tabs, types, bulk = util.small_bank(75, max(n, 1), n_branch=2, tpb=2, apt=5)
    bulk = wl.Bulk(bulk.type[:n], bulk.params[:, :n], bulk.ts[:n])
    s, g_tabs, g_st, g_res, key = run_relaxed(tabs, types, bulk, 3, strategy)
    assert s.error == 0
    if n:
        check_serializable(tabs, types, bulk, 3, g_tabs, g_st, g_res, key)
    assert s.committed == n


def test_relaxed_rejects_other_strategies():
    import torch
    from paper_1103_3105_amd import gputx
    tabs, types, bulk = util.small_bank(76, 10)
    eng = gputx.Engine(tabs, types)
    try:
        for strat in (gputx.AUTO, gputx.KSET):
            with pytest.raises(gputx.GputxError) as ei:
                eng.execute_relaxed(eng.bulk_to_device(bulk), strat, 3)
            assert ei.value.code == gputx.E_ARG
        torch.cuda.synchronize()
    finally:
        eng.close()
