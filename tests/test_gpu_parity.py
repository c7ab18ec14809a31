"""Bit-exact parity of the HIP engine with the serial oracle (GPU).

Every case runs the same seeded bulk through ``gputx_execute_bulk`` and
through the oracle and compares final tables (appended rows included),
per-transaction status and results element by element, plus the Appendix D
features against the Python references.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from oracle import reference as ref
from paper_1103_3105_amd import workloads as wl
from tests import util

pytestmark = pytest.mark.gpu

STRATS = ["TPL", "PART", "KSET", "AUTO"]


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def run_both(tabs, types, bulk, width, strategy, ts_sorted=False, **opts):
    import torch
    from paper_1103_3105_amd import gputx
    eng = gputx.Engine(tabs, types, **opts)
    try:
        dev = eng.bulk_to_device(bulk)
        st, res, stats = eng.execute(dev, gputx.STRATEGY[strategy], width, ts_sorted=ts_sorted)
        torch.cuda.synchronize()
        s = gputx.stats_from(stats)
        g_tabs = util.copy_tables(tabs)
        for name, t in g_tabs.items():
            host = eng.table_host(name)
            for c in range(len(t.cols)):
                t.cols[c][:] = host[c]
            if t.append:
                t.n_rows = eng.row_count(name)
        g_st = st.cpu().numpy()[:bulk.n]
        g_res = res.cpu().numpy()[:bulk.n]
    finally:
        eng.close()
    o_tabs = util.copy_tables(tabs)
    rc, o_st, o_res = oracle.run_serial(o_tabs, types, bulk.type, bulk.params, bulk.ts, width)
    return s, (g_tabs, g_st, g_res), (rc, o_tabs, o_st, o_res)


def assert_parity(s, g, o, bulk):
    g_tabs, g_st, g_res = g
    rc, o_tabs, o_st, o_res = o
    assert rc == 0 and s.error == 0, (rc, s.as_dict())
    ok, msg = util.tables_equal(o_tabs, g_tabs)
    assert ok, msg
    bad = np.flatnonzero(o_st != g_st)
    assert bad.size == 0, f"status differs at {bad[:8].tolist()}"
    bad = np.flatnonzero((o_res != g_res).any(axis=1))
    assert bad.size == 0, f"results differ at {bad[:8].tolist()}: {o_res[bad[:2]]} vs {g_res[bad[:2]]}"
    assert s.committed == int((o_st == 0).sum()) and s.aborted == int((o_st == 1).sum())
    assert s.invalid == int((o_st == 2).sum())


def check_features(s, tabs, types, bulk, part_size=1):
    per = ref.bulk_ops(types, bulk.type, bulk.params, bulk.ts, util.sizes_of(tabs),
                       util.roots_of(tabs))
    txn_ops = [o for _, _, o in per]
    w0, d, c = ref.features(txn_ops, util.roots_of(tabs), part_size)
    assert (s.w0, s.depth, s.cross) == (w0, d, c)
    assert s.n_ops == sum(len(o) for o in txn_ops)
    if s.chosen == 3:  # K-SET ran: one wave per k-set
        depth = ref.depth_scan(txn_ops)
        live = np.array([len(o) > 0 for o in txn_ops], dtype=bool)
        assert s.waves == (int(depth[live].max()) + 1 if live.any() else 0)


@pytest.mark.parametrize("strategy", STRATS)
@pytest.mark.parametrize("root_key", [False, True])
def test_config1_tiny_bank(strategy, root_key):
    w = wl.config1(root_key=root_key)
    _say("config1", strategy, root_key)
    s, g, o = run_both(w.tables, w.types, w.bulks[0], 3, strategy, ts_sorted=True)
    assert_parity(s, g, o, w.bulks[0])
    check_features(s, w.tables, w.types, w.bulks[0])
    if strategy == "KSET":
        assert s.waves == 4096


@pytest.mark.parametrize("strategy", STRATS)
@pytest.mark.parametrize("order", ["sorted", "shuffled", "gapped"])
def test_bank_multi_tile(strategy, order):
    tabs, types, bulk = util.small_bank(21, 20_000, n_branch=8, tpb=10, apt=300, theta=0.8)
    if order != "sorted":
        bulk = wl.shuffled(bulk, np.random.default_rng(5), gapped=order == "gapped")
    _say("bank", strategy, order)
    s, g, o = run_both(tabs, types, bulk, 3, strategy, ts_sorted=order == "sorted")
    assert_parity(s, g, o, bulk)
    check_features(s, tabs, types, bulk)


@pytest.mark.parametrize("strategy", STRATS)
def test_order_entry(strategy):
    tabs, types, bulk = util.small_order(22, 20_000, n_wh=4, d_per_w=10, c_per_d=30, items_per_w=500)
    _say("order", strategy)
    s, g, o = run_both(tabs, types, bulk, 16, strategy)
    assert_parity(s, g, o, bulk)
    check_features(s, tabs, types, bulk)


@pytest.mark.parametrize("strategy", STRATS)
def test_subscriber_with_aborts(strategy):
    tabs, types, bulk = util.small_sub(23, 20_000, n_sub=2000, theta=0.8)
    _say("subscriber", strategy)
    s, g, o = run_both(tabs, types, bulk, 14, strategy, part_size=16)
    assert_parity(s, g, o, bulk)
    assert s.aborted > 0
    check_features(s, tabs, types, bulk, part_size=16)


@pytest.mark.parametrize("scan", [1, 0])
@pytest.mark.parametrize("pipeline", [0, 1])
@pytest.mark.parametrize("workload", ["bank", "order", "sub"])
def test_part_forms(workload, pipeline, scan):
    """Both PART kernels: one wave per partition, and the pipelined pair of
    waves whose LDS cell table persists across chunks (the order and
    subscriber bulks fill it within a few chunks, so it is flushed often)."""
    if workload == "bank":
        tabs, types, bulk = util.small_bank(61, 20_000, n_branch=8, tpb=10, apt=300, theta=0.8)
        width, ps = 3, 1
    elif workload == "order":
        tabs, types, bulk = util.small_order(62, 20_000, n_wh=4, d_per_w=10, c_per_d=30,
                                             items_per_w=500)
        width, ps = 16, 1
    else:
        tabs, types, bulk = util.small_sub(63, 20_000, n_sub=2000, theta=0.8)
        width, ps = 14, 16
    _say("part form", workload, pipeline, scan)
    s, g, o = run_both(tabs, types, bulk, width, "PART", part_size=ps, part_pipeline=pipeline,
                       part_scan=scan)
    assert s.chosen == 2, s.as_dict()
    assert_parity(s, g, o, bulk)
    # transactions run side by side only when the scan form is enabled: the
    # bank's chunks as windows of one procedure, order entry's and the
    # subscribers' mixed chunks as runs of payments and reads, new-order
    # groups and subscriber-read groups
    if not scan:
        assert s.part_scan == 0
    else:
        assert s.part_scan > 0


@pytest.mark.parametrize("pipeline", [0, 1])
def test_part_partition_lengths(pipeline):
    """Partitions of 1, 31, 32, 33, 64, 65 and 200 transactions in one bulk
    (interleaved in timestamp order): the short ones run one per lane, the
    long ones (32 and more) one per workgroup with the LDS cell table."""
    counts = [1, 31, 32, 33, 64, 65, 200]
    nb, tpb, apt = len(counts), 3, 4
    rng = np.random.default_rng(64)
    n = sum(counts)
    tabs = wl.bank_tables(rng, nb, nb * tpb, nb * tpb * apt, history_capacity=n)
    branch = np.repeat(np.arange(nb), counts)
    rng.shuffle(branch)
    teller = branch * tpb + rng.integers(0, tpb, n)
    acct = teller * apt + rng.integers(0, apt, n)
    delta = rng.integers(-99_999, 100_000, n)
    bulk = wl.Bulk(np.zeros(n, np.int32), np.stack([acct, teller, branch, delta]).astype(np.int64),
                   np.arange(n, dtype=np.int64))
    _say("part lengths", pipeline)
    s, g, o = run_both(tabs, wl.bank_types(), bulk, 3, "PART", part_pipeline=pipeline)
    assert s.chosen == 2, s.as_dict()
    assert_parity(s, g, o, bulk)


@pytest.mark.parametrize("scan", [1, 0])
@pytest.mark.parametrize("pipeline", [0, 1])
@pytest.mark.parametrize("proc", ["PAYMENT", "ORDER_STATUS", "GET_SUB", "GET_CF",
                                  "UPD_SUB_FIELD", "UPD_LOC"])
def test_part_cellwise_one_procedure(proc, pipeline, scan):
    """Bulks of one cellwise procedure, so PART runs every chunk through the
    window form (a scan over each cell's maps).  Hot keys put many
    transactions on the same cells within a window: warehouse and district
    rows under payment, a few hundred Zipf(0.99) subscribers under the
    subscriber procedures, whose updates overwrite (maps with no old-value
    term)."""
    rng = np.random.default_rng(67)
    n = 20_000
    if proc in ("PAYMENT", "ORDER_STATUS"):
        mix = (0.0, 1.0, 0.0) if proc == "PAYMENT" else (0.0, 0.0, 1.0)
        bulk = wl.order_bulk(rng, n, 4, 10, 30, 500, mix=mix)
        tabs = wl.order_tables(rng, 4, 10, 30, 500, 1, 1)
        types, width, ps = wl.order_types(), 16, 1
    else:
        kinds = ["GET_SUB", "GET_CF", "UPD_SUB_FIELD", "UPD_LOC"]
        mix = tuple(1.0 if kinds[i] == proc else 0.0 for i in range(4)) + (0.0, 0.0)
        tabs = wl.sub_tables(rng, 300, occupancy=0.5)
        bulk = wl.sub_bulk(rng, n, 300, 0.99, mix=mix)
        types, width, ps = wl.sub_types(), 14, 16
    _say("part cellwise", proc, pipeline, scan)
    s, g, o = run_both(tabs, types, bulk, width, "PART", part_size=ps, part_pipeline=pipeline,
                       part_scan=scan)
    assert s.chosen == 2, s.as_dict()
    assert_parity(s, g, o, bulk)
    if not scan:
        assert s.part_scan == 0


@pytest.mark.parametrize("scan", [1, 0])
@pytest.mark.parametrize("pipeline", [0, 1])
@pytest.mark.parametrize("hot", [False, True])
def test_part_chunk_and_window_edges(pipeline, hot, scan):
    """Partitions of 255, 256, 257, 511, 513 and 769 debit-credits: around
    the 256-transaction chunks and 64-transaction windows.  hot: every
    transaction of a partition names the same account, teller and branch, so
    every window is one group per ordinal (the scan's longest groups)."""
    counts = [255, 256, 257, 511, 513, 769]
    nb, tpb, apt = len(counts), 3, 4
    rng = np.random.default_rng(68)
    n = sum(counts)
    tabs = wl.bank_tables(rng, nb, nb * tpb, nb * tpb * apt, history_capacity=n)
    branch = np.repeat(np.arange(nb), counts)
    rng.shuffle(branch)
    if hot:
        teller = branch * tpb
        acct = teller * apt
    else:
        teller = branch * tpb + rng.integers(0, tpb, n)
        acct = teller * apt + rng.integers(0, apt, n)
    delta = rng.integers(-99_999, 100_000, n)
    bulk = wl.Bulk(np.zeros(n, np.int32), np.stack([acct, teller, branch, delta]).astype(np.int64),
                   np.arange(n, dtype=np.int64))
    _say("part edges", pipeline, hot, scan)
    s, g, o = run_both(tabs, wl.bank_types(), bulk, 3, "PART", part_pipeline=pipeline,
                       part_scan=scan)
    assert s.chosen == 2, s.as_dict()
    assert_parity(s, g, o, bulk)


@pytest.mark.parametrize("pipeline", [0, 1])
def test_part_mixed_type_ids(pipeline):
    """Debit-credit registered under two type ids: chunks are not of one type,
    so PART runs them through its generic serial path (which checks that every
    cell a procedure names was staged) instead of the specialised one."""
    tabs, _, bulk = util.small_bank(65, 20_000, n_branch=8, tpb=10, apt=300, theta=0.8)
    types = [wl.TypeDesc(0, "DEBIT_CREDIT", 4, 3, wl.BANK_ROLES),
             wl.TypeDesc(1, "DEBIT_CREDIT", 4, 3, wl.BANK_ROLES)]
    typ = np.random.default_rng(66).integers(0, 2, bulk.n).astype(np.int32)
    bulk = wl.Bulk(typ, bulk.params, bulk.ts)
    _say("part mixed type ids", pipeline)
    s, g, o = run_both(tabs, types, bulk, 3, "PART", part_pipeline=pipeline)
    assert s.chosen == 2, s.as_dict()
    assert_parity(s, g, o, bulk)


@pytest.mark.parametrize("n", [0, 1, 2, 63, 4097])
def test_small_and_empty_bulks(n):
    tabs, types, bulk = util.small_bank(24, max(n, 1), n_branch=2, tpb=2, apt=5)
    if n == 0:
        bulk = wl.Bulk(bulk.type[:0], bulk.params[:, :0], bulk.ts[:0])
    _say("small", n)
    for strategy in STRATS:
        s, g, o = run_both(tabs, types, bulk, 3, strategy)
        assert_parity(s, g, o, bulk)


def test_invalid_transactions():
    tabs, types, bulk = util.small_bank(25, 5000, n_branch=4, tpb=4, apt=10)
    bulk.params[0, ::7] = 10**9
    bulk.type[::11] = 9
    bulk.params[2, ::13] = -5
    for strategy in STRATS:
        s, g, o = run_both(tabs, types, bulk, 3, strategy)
        assert_parity(s, g, o, bulk)
        assert s.invalid > 0


def test_duplicate_timestamp_is_bulk_error():
    from paper_1103_3105_amd import gputx
    tabs, types, bulk = util.small_bank(26, 3000)
    bulk.ts[100] = bulk.ts[2000]
    for ts_sorted in (False,):
        s, g, o = run_both(tabs, types, bulk, 3, "AUTO", ts_sorted=ts_sorted)
        assert s.error == gputx.E_DUP_TS and o[0] == oracle.E_DUP_TS
        ok, msg = util.tables_equal(tabs, g[0])
        assert ok, msg
    bulk2 = util.small_bank(27, 3000)[2]
    bulk2.ts[10] = bulk2.ts[11]   # adjacent duplicate in ascending input
    s, g, o = run_both(tabs, types, bulk2, 3, "KSET", ts_sorted=True)
    assert s.error == gputx.E_DUP_TS
    ok, _ = util.tables_equal(tabs, g[0])
    assert ok


def test_unsorted_flagged_sorted_is_error():
    from paper_1103_3105_amd import gputx
    tabs, types, bulk = util.small_bank(28, 3000)
    bulk = wl.shuffled(bulk, np.random.default_rng(1))
    s, g, o = run_both(tabs, types, bulk, 3, "TPL", ts_sorted=True)
    assert s.error == gputx.E_UNSORTED
    ok, _ = util.tables_equal(tabs, g[0])
    assert ok


def test_append_capacity_error_writes_nothing_past_capacity():
    """An overflowing bulk leaves even the rows past the declared capacity
    untouched, under every strategy (the columns here are longer than the
    capacity the table declares, so a stray append would land in them)."""
    from paper_1103_3105_amd import gputx
    tabs, types, bulk = util.small_bank(30, 3000)
    tabs["history"] = wl.Table("history", ["i64"] * 5, [np.zeros(4096, np.int64) for _ in range(5)],
                               0, 100, append=True)
    for strategy in STRATS:
        s, g, o = run_both(tabs, types, bulk, 3, strategy)
        assert s.error == gputx.E_CAPACITY and o[0] == oracle.E_CAPACITY, strategy
        for c in g[0]["history"].cols:
            assert not c.any(), strategy
        ok, msg = util.tables_equal(tabs, g[0])
        assert ok, (strategy, msg)


def test_append_capacity_error():
    from paper_1103_3105_amd import gputx
    tabs, types, bulk = util.small_bank(29, 3000)
    tabs["history"] = wl.Table("history", ["i64"] * 5, [np.zeros(100, np.int64) for _ in range(5)],
                               0, 100, append=True)
    s, g, o = run_both(tabs, types, bulk, 3, "PART")
    assert s.error == gputx.E_CAPACITY and o[0] == oracle.E_CAPACITY
    ok, _ = util.tables_equal(tabs, g[0])
    assert ok


# ---------------------------------------------------------------------------
# cross-partition transactions and Algorithm 1's branches

def _remote_bank(seed, n=20_000, remote_frac=0.05, theta=0.8):
    rng = np.random.default_rng(seed)
    tabs = wl.bank_tables(rng, 8, 80, 24_000, history_capacity=n)
    bulk = wl.bank_bulk(rng, n, 8, 80, 24_000, theta, remote_frac=remote_frac)
    return tabs, wl.bank_types(), bulk


@pytest.mark.parametrize("strategy", STRATS)
def test_cross_partition_bulk(strategy):
    """A bank bulk where about 5% of debit-credits use a teller of another
    branch (c > 0).  PART, requested or picked by Algorithm 1, hands the
    bulk to TPL (Section 5.2); every strategy stays bit-exact, appended
    history rows included."""
    tabs, types, bulk = _remote_bank(31)
    _say("cross-partition bank", strategy)
    s, g, o = run_both(tabs, types, bulk, 3, strategy, ts_sorted=True)
    assert_parity(s, g, o, bulk)
    check_features(s, tabs, types, bulk)
    assert s.cross > 0
    want = {"TPL": 1, "PART": 1, "KSET": 3, "AUTO": 1}[strategy]
    assert s.chosen == want, s.as_dict()


def test_cross_partition_hand_built_bulk():
    """The six-transaction hand-counted case of the oracle pins (c = 2)."""
    rng = np.random.default_rng(77)
    tabs = wl.bank_tables(rng, 2, 4, 12, history_capacity=8)
    p = np.array([[0, 7, 1, 11, 5, 6], [0, 3, 2, 1, 1, 2], [0, 1, 1, 0, 0, 1],
                  [10, -20, 30, -40, 50, -60]], dtype=np.int64)
    bulk = wl.Bulk(np.zeros(6, np.int32), p, np.arange(6, dtype=np.int64))
    for strategy in ("PART", "AUTO"):
        s, g, o = run_both(tabs, wl.bank_types(), bulk, 3, strategy, ts_sorted=True)
        assert_parity(s, g, o, bulk)
        assert (s.cross, s.w0, s.chosen) == (2, 2, 1), s.as_dict()


@pytest.mark.parametrize("remote", [0.0, 0.05])
@pytest.mark.parametrize("bars", [
    dict(w0_bar=1, c_bar=0, d_bar=1 << 30),            # K-SET: w0 >= w0_bar
    dict(w0_bar=1 << 40, c_bar=1 << 40, d_bar=1 << 30),  # PART: c <= c_bar
    dict(w0_bar=1 << 40, c_bar=-1, d_bar=1),           # PART: d >= d_bar
    dict(w0_bar=1 << 40, c_bar=-1, d_bar=1 << 30),     # TPL
])
def test_algorithm1_choice_matches_reference(bars, remote):
    """Algorithm 1 on the device takes the branch the reference rule takes
    for the bulk's own (w0, d, c), followed by Section 5.2's PART -> TPL
    hand-off when c > 0; the chosen executor is bit-exact."""
    tabs, types, bulk = _remote_bank(32, n=6000, remote_frac=remote)
    s, g, o = run_both(tabs, types, bulk, 3, "AUTO", ts_sorted=True, **bars)
    assert_parity(s, g, o, bulk)
    per = ref.bulk_ops(types, bulk.type, bulk.params, bulk.ts, util.sizes_of(tabs),
                       util.roots_of(tabs))
    w0, d, c = ref.features([x for _, _, x in per], util.roots_of(tabs), 1)
    pick = ref.choose_strategy(w0, d, c, bars["w0_bar"], bars["c_bar"], bars["d_bar"])
    want = ref.strategy_run(pick, c)
    assert gputx_name(s.chosen) == want, (s.as_dict(), pick, want)


def gputx_name(code):
    from paper_1103_3105_amd import gputx
    return gputx.STRATEGY_NAME[code]


# ---------------------------------------------------------------------------
# a type that is not two-phase: new-orders that roll back from an undo log

@pytest.mark.parametrize("strategy", STRATS)
def test_order_entry_with_rollbacks(strategy):
    """5% of new-orders name the unused item after updating the stock of
    their earlier items and roll those updates back (Appendix D's undo
    logging); every executor leaves exactly the serial result."""
    tabs, types, bulk = util.small_order(25, 20_000, n_wh=4, d_per_w=10, c_per_d=30, items_per_w=500,
                                         rollback_frac=0.05)
    _say("order with rollbacks", strategy)
    s, g, o = run_both(tabs, types, bulk, 16, strategy)
    assert_parity(s, g, o, bulk)
    check_features(s, tabs, types, bulk)
    assert s.aborted > 100


@pytest.mark.parametrize("pipeline", [0, 1])
def test_part_forms_with_rollbacks(pipeline):
    """PART's LDS cell tables: the rollback restores the staged values."""
    tabs, types, bulk = util.small_order(26, 20_000, n_wh=2, d_per_w=10, c_per_d=30, items_per_w=100,
                                         rollback_frac=0.2)
    s, g, o = run_both(tabs, types, bulk, 16, "PART", part_pipeline=pipeline)
    assert s.chosen == 2
    assert_parity(s, g, o, bulk)
    assert s.aborted > 100


@pytest.mark.parametrize("strategy", ["PART", "TPL", "KSET"])
@pytest.mark.parametrize("rollback", [0.0, 0.1])
def test_order_entry_repeated_items(strategy, rollback):
    """New-orders naming an item twice update that stock row twice in a row
    (PART's wave-wide form falls back to one lane for them); with rollbacks,
    the undo log restores the row through both updates."""
    tabs, types, bulk = util.small_order(27, 8000, n_wh=2, d_per_w=10, c_per_d=30, items_per_w=100,
                                         rollback_frac=rollback)
    no = np.flatnonzero(bulk.type == 1)
    rng = np.random.default_rng(28)
    rep = no[rng.random(no.size) < 0.3]
    prm = bulk.params.copy()
    prm[5, rep] = prm[4, rep]          # second item = first item
    bulk = wl.Bulk(bulk.type, prm, bulk.ts)
    s, g, o = run_both(tabs, types, bulk, 16, strategy)
    assert_parity(s, g, o, bulk)


@pytest.mark.parametrize("pipeline", [0, 1])
@pytest.mark.parametrize("mix", [(0.0, 0.5, 0.5), (0.3, 0.4, 0.3)])
def test_part_mixed_windows(pipeline, mix):
    """A serial wave's run of payments and order-status reads executes as one
    window over their cell accesses, grouped by cell.  Two customers per
    district make a read often the last access of a customer's group, after
    payments to it in the same window: the cell must keep their sum."""
    rng = np.random.default_rng(32)
    n = 12_000
    bulk = wl.order_bulk(rng, n, 2, 4, 2, 300, mix=mix)
    n_no = int((bulk.type == 1).sum())
    n_l = int(bulk.params[3][bulk.type == 1].sum())
    tabs = wl.order_tables(rng, 2, 4, 2, 300, max(n_no, 1), max(n_l, 1))
    _say("mixed windows", pipeline, mix)
    s, g, o = run_both(tabs, wl.order_types(), bulk, 16, "PART", part_pipeline=pipeline)
    assert s.chosen == 2
    assert_parity(s, g, o, bulk)


@pytest.mark.parametrize("pipeline", [0, 1])
@pytest.mark.parametrize("rollback", [0.0, 0.02])
def test_part_new_order_groups(pipeline, rollback):
    """New-orders over a large item space rarely share a stock row, so PART's
    serial wave runs them four at a time (sixteen lanes each); a group in
    which two items meet, or a new-order rolls back, runs one at a time.  A
    few planted repeats and shared items exercise both within the same
    chunks."""
    tabs, types, bulk = util.small_order(29, 30_000, n_wh=3, d_per_w=10, c_per_d=30, items_per_w=100_000,
                                         rollback_frac=rollback)
    no = np.flatnonzero(bulk.type == 1)
    rng = np.random.default_rng(30)
    prm = bulk.params.copy()
    rep = no[rng.random(no.size) < 0.02]
    prm[5, rep] = prm[4, rep]                  # an item named twice in one new-order
    nxt = no[1:][rng.random(no.size - 1) < 0.02]
    prm[4, nxt] = prm[4, nxt - 1]              # an item of the transaction before (if it is a new-order)
    bulk = wl.Bulk(bulk.type, prm, bulk.ts)
    _say("new-order groups", pipeline, rollback)
    s, g, o = run_both(tabs, types, bulk, 16, "PART", part_pipeline=pipeline)
    assert s.chosen == 2
    assert_parity(s, g, o, bulk)


@pytest.mark.parametrize("lanes", [0, 1, 3, 16, 64])
@pytest.mark.parametrize("workload", ["bank", "order", "sub"])
def test_tpl_window_shapes(workload, lanes):
    """TPL with per-wave windows of `lanes` transactions (the other lanes
    idle) gives the serial result on skewed bank, order entry with rollbacks
    and repeated items, and the subscriber mix with aborts; a ragged last
    window included (sizes not a multiple of the window)."""
    if workload == "bank":
        tabs, types, bulk = util.small_bank(61, 20_001, n_branch=8, tpb=10, apt=300, theta=0.9)
        width, opts = 3, {}
    elif workload == "order":
        tabs, types, bulk = util.small_order(62, 6_007, n_wh=2, d_per_w=10, c_per_d=30, items_per_w=40,
                                             rollback_frac=0.1)
        width, opts = 16, {}
    else:
        tabs, types, bulk = util.small_sub(63, 20_003, n_sub=2000, theta=0.8)
        width, opts = 14, dict(part_size=16)
    _say("tpl shape", workload, lanes)
    s, g, o = run_both(tabs, types, bulk, width, "TPL", tpl_lanes=lanes, **opts)
    assert s.chosen == 1
    assert_parity(s, g, o, bulk)


def test_part_size_sweep_and_tuning():
    """PART at several partition sizes (root keys per partition, Section
    5.2's tuning parameter) gives the serial result each time, and the
    calibration returns one of the candidates with a time for each."""
    from paper_1103_3105_amd import autotune
    tabs, types, bulk = util.small_sub(64, 8_000, n_sub=2000, theta=0.8)
    for size in (1, 16, 256):
        _say("part size", size)
        s, g, o = run_both(tabs, types, bulk, 14, "PART", part_size=size)
        assert_parity(s, g, o, bulk)
    tuned = autotune.tune_part_size(tabs, types, [(bulk, 14, 0)], sizes=(1, 16, 256))
    assert tuned["best"] in (1, 16, 256)
    assert set(tuned["ms"]) == {1, 16, 256} and all(v > 0 for v in tuned["ms"].values())


def test_type_mask_layout_and_exclusion():
    """A context with order entry and debit-credit registered: a bank bulk
    whose type mask names debit-credit alone runs with debit-credit's PART
    layout and gives the serial result; a mask that leaves a present type out
    makes that type's transactions INVALID (and the rest still serial)."""
    import torch
    from paper_1103_3105_amd import batching, gputx
    bw = batching.config4(n_bulks=6, lo=2048, hi=4096, repeats=1, bank_branches=8,
                          accounts_per_branch=1000, n_wh=4, items_per_w=1000, c_per_d=30)
    db, bulk = next((d, b) for d, b in bw.jobs if d == "bank")
    eng = gputx.Engine(bw.tables, bw.types)
    try:
        dev = eng.bulk_to_device(bulk)
        want_mask = int(np.bitwise_or.reduce(np.left_shift(1, np.unique(bulk.type))))
        assert dev["type_mask"] == want_mask
        st, res, stats = eng.execute(dev, gputx.STRATEGY["PART"], batching.WIDTH[db], ts_sorted=True)
        torch.cuda.synchronize()
        s = gputx.stats_from(stats)
        g_st, g_res = st.cpu().numpy()[:bulk.n], res.cpu().numpy()[:bulk.n]
    finally:
        eng.close()
    o_tabs = util.copy_tables(bw.tables)
    rc, o_st, o_res = oracle.run_serial(o_tabs, bw.types, bulk.type, bulk.params, bulk.ts, batching.WIDTH[db])
    assert rc == 0 and s.error == 0
    assert np.array_equal(g_st, o_st) and np.array_equal(g_res, o_res)
    # leave the bulk's only type out of the mask (keep another registered type)
    other = next(t.type_id for t in bw.types if t.type_id not in set(np.unique(bulk.type).tolist()))
    eng = gputx.Engine(bw.tables, bw.types)
    try:
        dev = eng.bulk_to_device(bulk)
        dev["type_mask"] = 1 << other
        st, res, stats = eng.execute(dev, gputx.STRATEGY["AUTO"], batching.WIDTH[db], ts_sorted=True)
        torch.cuda.synchronize()
        s = gputx.stats_from(stats)
        assert s.error == 0 and s.invalid == bulk.n and s.committed == 0
        assert np.all(st.cpu().numpy()[:bulk.n] == 2)
    finally:
        eng.close()
