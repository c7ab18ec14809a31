"""Pins of the serial oracle and the dependency references against what the
paper and the mathematics fix (CPU only)."""
from __future__ import annotations

import os

import numpy as np
import pytest

import oracle
from oracle import reference as ref
from paper_1103_3105_amd import workloads as wl
from tests import util

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = {}
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            rows.setdefault(key, []).append(vals)
    return rows


# ---------------------------------------------------------------------------
# Section 4: rank rule, depth, k-sets

def test_fig1_group_a_ranks_and_ksets():
    g = _read_golden("fig1_group_a.txt")
    ops = g["ops"][0]
    txn_ops = [{("a", 0): o == "W"} for o in ops]
    flat, ranks, maxrank = ref.paper_ranks(txn_ops)
    assert ranks.tolist() == [int(x) for x in g["ranks"][0]]
    want = {int(k[0]): sorted(int(t[1:]) - 1 for t in k[1:]) for k in g["kset"]}
    for depth in (ref.depth_pairwise(txn_ops), ref.depth_appendix_b(txn_ops),
                  ref.depth_scan(txn_ops)):
        got = {}
        for t, d in enumerate(depth):
            got.setdefault(int(d), []).append(t)
        assert got == want
    assert ref.kahn_levels(txn_ops) == [want[k] for k in sorted(want)]
    edges = ref.tdg_edges_pairwise(txn_ops)
    a, b = (int(x[1:]) - 1 for x in g["no_edge"][0])
    assert (a, b) not in edges and ref.conflict(txn_ops[a], txn_ops[b])
    assert sorted(edges) == [(0, 1), (0, 2), (1, 3), (2, 3)]


def test_rank_is_not_depth_counterexample():
    # T1 = {W a}, T2 = {W a, W b}, T3 = {W b}: T2 and T3 conflict, so they
    # cannot share a k-set (Property 1) although both have maximum rank 1.
    txn_ops = [{("a", 0): True}, {("a", 0): True, ("b", 0): True}, {("b", 0): True}]
    _, _, maxrank = ref.paper_ranks(txn_ops)
    assert maxrank.tolist() == [0, 1, 1]
    assert ref.depth_scan(txn_ops).tolist() == [0, 1, 2]
    assert ref.depth_pairwise(txn_ops).tolist() == [0, 1, 2]


def _random_txn_ops(rng, n, n_items, max_ops, p_write):
    out = []
    for _ in range(n):
        k = int(rng.integers(1, max_ops + 1))
        ops = {}
        for it in rng.integers(0, n_items, k):
            ops[("x", int(it))] = ops.get(("x", int(it)), False) or bool(rng.random() < p_write)
        out.append(ops)
    return out


@pytest.mark.parametrize("seed", range(40))
def test_depth_methods_agree_and_properties(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 40))
    txn_ops = _random_txn_ops(rng, n, int(rng.integers(1, 12)), 4, float(rng.random()))
    d1 = ref.depth_pairwise(txn_ops)
    d2 = ref.depth_appendix_b(txn_ops)
    d3 = ref.depth_scan(txn_ops)
    assert np.array_equal(d1, d2) and np.array_equal(d1, d3)
    levels = ref.kahn_levels(txn_ops)
    for k, lvl in enumerate(levels):
        assert all(d1[t] == k for t in lvl)
        # Property 1: a k-set is conflict-free
        for i in range(len(lvl)):
            for j in range(i + 1, len(lvl)):
                assert not ref.conflict(txn_ops[lvl[i]], txn_ops[lvl[j]])
        # Property 2: each member of a k-set (k >= 1) conflicts with one of the (k-1)-set
        if k:
            for t in lvl:
                assert any(ref.conflict(txn_ops[u], txn_ops[t]) for u in levels[k - 1])
    assert sum(len(l) for l in levels) == n
    _, _, maxrank = ref.paper_ranks(txn_ops)
    assert np.all(maxrank <= d1)
    assert np.array_equal(maxrank == 0, d1 == 0)      # the 0-set is exact


@pytest.mark.parametrize("seed", range(10))
def test_single_op_rank_equals_depth(seed):
    rng = np.random.default_rng(100 + seed)
    txn_ops = _random_txn_ops(rng, 60, 5, 1, 0.4)
    _, _, maxrank = ref.paper_ranks(txn_ops)
    assert np.array_equal(maxrank, ref.depth_scan(txn_ops))


def test_tpcb_root_key_closed_form():
    # Section 5.1 / Figure 2: with the lock on the branch, the T-dependency
    # graph is one path per branch and the key of a k-set member is k.
    tabs, _, bulk = util.small_bank(7, 300, n_branch=5, tpb=3, apt=4, theta=0.0)
    types = wl.bank_types(root_key=True)
    per = ref.bulk_ops(types, bulk.type, bulk.params, bulk.ts, util.sizes_of(tabs),
                       util.roots_of(tabs))
    txn_ops = [o for _, _, o in per]
    assert all(len(o) == 1 and list(o)[0][0] == "branch" for o in txn_ops)
    branch = bulk.params[2][np.argsort(bulk.ts)]
    earlier = np.array([(branch[:i] == branch[i]).sum() for i in range(len(branch))])
    _, _, maxrank = ref.paper_ranks(txn_ops)
    assert np.array_equal(maxrank, earlier)
    assert np.array_equal(ref.depth_scan(txn_ops), earlier)


def test_config1_depth_and_zero_set():
    w = wl.config1()
    b = w.bulks[0]
    per = ref.bulk_ops(w.types, b.type, b.params, b.ts, util.sizes_of(w.tables),
                       util.roots_of(w.tables))
    txn_ops = [o for _, _, o in per]
    depth = ref.depth_scan(txn_ops)
    assert depth.max() == 4095 and np.array_equal(depth, np.arange(4096))
    w0, d, c = ref.features(txn_ops, util.roots_of(w.tables), 1)
    assert (w0, d, c) == (1, 4095, 0)


def test_alg1_truth_table():
    cases = [
        ((100, 5, 3), "KSET"), ((99, 5, 0), "PART"), ((99, 50, 3), "PART"),
        ((99, 5, 3), "TPL"), ((100, 50, 50), "KSET"), ((0, 9, 1), "TPL"), ((0, 10, 1), "PART"),
    ]
    for (w0, d, c), want in cases:
        assert ref.choose_strategy(w0, d, c, w0_bar=100, c_bar=0, d_bar=10) == want


def _cross_bank():
    """Hand-built bank: 2 branches x 2 tellers x 3 accounts, 6 debit-credits
    of which two go through a teller of the other branch (hand-counted)."""
    rng = np.random.default_rng(77)
    tabs = wl.bank_tables(rng, 2, 4, 12, history_capacity=8)
    #            acct  teller branch    account's branch   teller's branch
    rows = [(0, 0, 0),    # 0          0                  local
            (7, 3, 1),    # 1          1                  local
            (1, 2, 1),    # 0          1                  cross
            (11, 1, 0),   # 1          0                  cross
            (5, 1, 0),    # 0          0                  local
            (6, 2, 1)]    # 1          1                  local
    p = np.array([[a for a, _, _ in rows], [t for _, t, _ in rows], [b for _, _, b in rows],
                  [10, -20, 30, -40, 50, -60]], dtype=np.int64)
    bulk = wl.Bulk(np.zeros(6, np.int32), p, np.arange(6, dtype=np.int64))
    return tabs, wl.bank_types(), bulk


def test_cross_partition_count_hand_counted():
    """Appendix D's c: transactions whose items lie under more than one
    partition root.  Two of the six cross branches; with both branches in
    one partition none does."""
    tabs, types, bulk = _cross_bank()
    per = ref.bulk_ops(types, bulk.type, bulk.params, bulk.ts, util.sizes_of(tabs),
                       util.roots_of(tabs))
    txn_ops = [o for _, _, o in per]
    roots = util.roots_of(tabs)
    assert [len(ref.partitions_of(o, roots, 1)) for o in txn_ops] == [1, 1, 2, 2, 1, 1]
    w0, d, c = ref.features(txn_ops, roots, 1)
    assert c == 2
    assert ref.features(txn_ops, roots, 2)[2] == 0
    # hand-counted w0: only t0 and t1 have no earlier conflicting txn (t2
    # meets t1 on branch 1, t3 meets t0 on branch 0, t4 meets t3 on teller 1,
    # t5 meets t2 on teller 2)
    assert w0 == 2
    # root-key locking: every op becomes its partition root; the cross txns
    # then name two roots
    per_r = ref.bulk_ops(wl.bank_types(root_key=True), bulk.type, bulk.params, bulk.ts,
                         util.sizes_of(tabs), roots)
    assert [len(o) for _, _, o in per_r] == [1, 1, 2, 2, 1, 1]
    # serial semantics still hold: final balances are initial + per-row sums
    t, st, _ = _run(tabs, types, bulk, 3)
    assert (st == 0).all()
    for role, col in (("account", 0), ("teller", 1), ("branch", 2)):
        want = tabs[role].cols[0].copy()
        np.add.at(want, bulk.params[col], bulk.params[3])
        assert np.array_equal(t[role].cols[0], want), role


def test_cross_partition_bulks_run_under_tpl():
    """Section 5.2: PART with a cross-partition transaction hands the bulk to
    TPL; Algorithm 1's own choice is unchanged otherwise."""
    assert ref.strategy_run("PART", 1) == "TPL"
    assert ref.strategy_run("PART", 0) == "PART"
    assert ref.strategy_run("KSET", 5) == "KSET"
    assert ref.strategy_run("TPL", 5) == "TPL"
    # Algorithm 1 with c > c_bar but d >= d_bar picks PART, which then runs as TPL
    assert ref.strategy_run(ref.choose_strategy(3, 50, 2, 100, 0, 10), 2) == "TPL"


def test_remote_generator_counts():
    """The generator's remote fraction yields cross-partition transactions at
    about that rate, and every remote teller lies in another branch."""
    rng = np.random.default_rng(5)
    b = wl.bank_bulk(rng, 20000, 8, 80, 8000, 0.0, remote_frac=0.15)
    acct_branch = b.params[0] // 1000
    cross = acct_branch != b.params[2]
    assert abs(cross.mean() - 0.15) < 0.02
    assert np.array_equal(b.params[2], b.params[1] // 10)


# ---------------------------------------------------------------------------
# serial semantics: closed forms and invariants

def _run(tabs, types, bulk, width):
    t = util.copy_tables(tabs)
    rc, st, res = oracle.run_serial(t, types, bulk.type, bulk.params, bulk.ts, width)
    assert rc == 0
    return t, st, res


@pytest.mark.parametrize("which", ["config1", "skewed"])
def test_debit_credit_closed_form(which):
    if which == "config1":
        w = wl.config1()
        tabs, types, bulk = w.tables, w.types, w.bulks[0]
    else:
        tabs, types, bulk = util.small_bank(3, 5000, n_branch=4, tpb=5, apt=50, theta=0.99)
    out, st, res = _run(tabs, types, bulk, 3)
    assert (st == 0).all()
    order = np.argsort(bulk.ts)
    acct, tel, br, d = (bulk.params[k][order] for k in range(4))
    for col, key, role in ((0, acct, "account"), (1, tel, "teller"), (2, br, "branch")):
        init = tabs[role].cols[0]
        post = init[key] + util.seg_inclusive_prefix(key, d)
        assert np.array_equal(res[order, col], post), role
        final = init.copy()
        np.add.at(final, key, d)
        assert np.array_equal(out[role].cols[0], final), role
        assert out[role].cols[0].sum() - init.sum() == d.sum()
    h = out["history"]
    assert h.n_rows == bulk.n
    for c, v in enumerate((acct, tel, br, d, bulk.ts[order])):
        assert np.array_equal(h.cols[c][:h.n_rows], v)


def test_input_order_and_gapped_timestamps():
    tabs, types, bulk = util.small_bank(4, 3000, n_branch=3, tpb=3, apt=20, theta=0.8)
    base, st0, res0 = _run(tabs, types, bulk, 3)
    rng = np.random.default_rng(9)
    for gapped in (False, True):
        sb = wl.shuffled(bulk, rng, gapped=gapped)
        out, st, res = _run(tabs, types, sb, 3)
        # same transactions (matched by parameters + rank of ts) give the same results
        o0 = np.argsort(bulk.ts)
        o1 = np.argsort(sb.ts)
        assert np.array_equal(res0[o0], res[o1]) and np.array_equal(st0[o0], st[o1])
        for role in ("account", "teller", "branch"):
            assert np.array_equal(base[role].cols[0], out[role].cols[0])
        assert np.array_equal(out["history"].cols[4][:bulk.n], np.sort(sb.ts))


def test_payment_and_order_status_closed_form():
    tabs, types, bulk = util.small_order(5, 4000, n_wh=3, d_per_w=4, c_per_d=5, items_per_w=60)
    out, st, res = _run(tabs, types, bulk, 16)
    assert (st == 0).all()
    order = np.argsort(bulk.ts)
    ty = bulk.type[order]
    w, d, c, h = (bulk.params[k][order] for k in range(4))
    drow = w * 4 + d
    crow = drow * 5 + c
    pay = ty == 2
    hh = np.where(pay, h, 0)
    for col, key, role in ((0, w, "warehouse"), (1, drow, "district"), (2, crow, "customer")):
        init = tabs[role].cols[0]
        post = init[key] + util.seg_inclusive_prefix(key, hh)
        assert np.array_equal(res[order][pay, col], post[pay]), role
        final = init.copy()
        np.add.at(final, key, hh)
        assert np.array_equal(out[role].cols[0], final)
    # order-status sees every earlier payment of its customer
    stat = ty == 3
    seen = tabs["customer"].cols[0][crow] + util.seg_inclusive_prefix(crow, hh)
    assert np.array_equal(res[order][stat, 0], seen[stat])


def test_new_order_stock_chain():
    tabs, types, bulk = util.small_order(6, 3000, n_wh=2, d_per_w=2, c_per_d=3, items_per_w=25)
    out, st, res = _run(tabs, types, bulk, 16)
    order = np.argsort(bulk.ts)
    stock = tabs["stock"].cols[0].astype(np.int64).copy()
    n_lines = 0
    wraps = 0
    qsum = 0
    lines = out["order_line"]
    for i in order:
        if bulk.type[i] != 1:
            continue
        p = bulk.params[:, i]
        k = int(p[3])
        assert res[i, 0] == k
        for j in range(k):
            row = p[0] * 25 + p[4 + j]
            prev, q, s = stock[row], int(p[19 + j]), int(res[i, 1 + j])
            assert s == prev - q or (s == prev - q + 91 and prev - q < 10)
            assert (s == prev - q + 91) == (prev - q < 10)
            wraps += int(prev - q < 10)
            qsum += q
            stock[row] = s
            assert tuple(c[n_lines] for c in lines.cols) == (bulk.ts[i], j, p[4 + j], q, p[0])
            n_lines += 1
    assert np.array_equal(out["stock"].cols[0], stock)
    s0, s1 = tabs["stock"].cols[0].astype(np.int64), out["stock"].cols[0].astype(np.int64)
    assert s1.sum() - s0.sum() == -qsum + 91 * wraps
    assert s1.min() >= 10 and s1.max() <= 100
    no = np.sort(bulk.ts[bulk.type == 1])
    assert out["orders"].n_rows == no.size and np.array_equal(out["orders"].cols[0][:no.size], no)
    assert lines.n_rows == n_lines


def test_subscriber_chains():
    tabs, types, bulk = util.small_sub(8, 3000, n_sub=7, theta=0.8)
    out, st, res = _run(tabs, types, bulk, 14)
    order = np.argsort(bulk.ts)
    sub = [c.astype(np.int64).copy() for c in tabs["subscriber"].cols]
    cf = [c.astype(np.int64).copy() for c in tabs["call_fwd"].cols]
    ins = dels = 0
    for i in order:
        ty, p = int(bulk.type[i]), bulk.params[:, i]
        slot = p[0] * 12 + p[1]
        if ty == 4:
            assert res[i].tolist() == [int(sub[1 + f][p[0]]) for f in range(14)]
        elif ty == 5:
            assert res[i, :3].tolist() == [int(cf[0][slot]), int(cf[1][slot]), int(cf[2][slot])]
        elif ty in (6, 7):
            col = 1 + p[1] + (4 if ty == 7 else 0)
            assert res[i, 0] == sub[col][p[0]]
            sub[col][p[0]] = p[2]
        elif ty == 8:
            assert (st[i] == 1) == bool(cf[0][slot])
            if st[i] == 0:
                cf[0][slot], cf[1][slot], cf[2][slot] = 1, p[2], p[3]
                ins += 1
        elif ty == 9:
            assert (st[i] == 1) == (not cf[0][slot])
            if st[i] == 0:
                assert res[i, :3].tolist() == [1, int(cf[1][slot]), int(cf[2][slot])]
                cf[0][slot] = cf[1][slot] = cf[2][slot] = 0
                dels += 1
    for c in range(15):
        assert np.array_equal(out["subscriber"].cols[c].astype(np.int64), sub[c])
    for c in range(3):
        assert np.array_equal(out["call_fwd"].cols[c].astype(np.int64), cf[c])
    d_occ = int(out["call_fwd"].cols[0].sum()) - int(tabs["call_fwd"].cols[0].sum())
    assert d_occ == ins - dels and ins > 0 and dels > 0


# ---------------------------------------------------------------------------
# brute force: every linear extension of the conflict order gives the serial result

def _mixed_tiny(seed, n):
    rng = np.random.default_rng(seed)
    kind = int(rng.integers(0, 4))
    if kind == 0:
        return util.small_bank(seed, n, n_branch=1, tpb=2, apt=2, theta=0.0), 3
    if kind == 1:
        return util.small_order(seed, n, n_wh=1, d_per_w=2, c_per_d=2, items_per_w=6), 16
    if kind == 3:   # new-orders that are not two-phase, half of them rolling back
        return util.small_order(seed, n, n_wh=1, d_per_w=2, c_per_d=2, items_per_w=6,
                                rollback_frac=0.5), 16
    return util.small_sub(seed, n, n_sub=2, theta=0.0), 14


@pytest.mark.parametrize("seed", range(24))
def test_bruteforce_linear_extensions(seed):
    n = 3 + seed % 5
    (tabs, types, bulk), width = _mixed_tiny(seed, n)
    sizes = util.sizes_of(tabs)
    per = ref.bulk_ops(types, bulk.type, bulk.params, bulk.ts, sizes, util.roots_of(tabs))
    txn_ops = [o for _, _, o in per]
    idx_of_pos = [i for i, _, _ in per]
    # the C oracle equals the Python twin in timestamp order, appends included
    c_tabs, c_st, c_res = _run(tabs, types, bulk, width)
    p_tabs = util.copy_tables(tabs)
    p_st, p_res = ref.py_execute(p_tabs, types, bulk.type, bulk.params, bulk.ts, width)
    ok, msg = util.tables_equal(c_tabs, p_tabs)
    assert ok, msg
    assert np.array_equal(c_st, p_st) and np.array_equal(c_res, p_res)
    n_ext = 0
    for ext in ref.linear_extensions(txn_ops):
        e_tabs = util.copy_tables(tabs)
        e_st, e_res = ref.py_execute(e_tabs, types, bulk.type, bulk.params, bulk.ts, width,
                                     order=[idx_of_pos[k] for k in ext])
        ok, msg = util.tables_equal(c_tabs, e_tabs, append_sort_col=0)
        assert ok, (ext, msg)
        assert np.array_equal(c_st, e_st) and np.array_equal(c_res, e_res), ext
        n_ext += 1
    assert n_ext >= 1


# ---------------------------------------------------------------------------
# error handling

def test_duplicate_timestamp_is_bulk_error_without_mutation():
    tabs, types, bulk = util.small_bank(11, 50)
    bulk.ts[7] = bulk.ts[30]
    t = util.copy_tables(tabs)
    rc, st, res = oracle.run_serial(t, types, bulk.type, bulk.params, bulk.ts, 3)
    assert rc == oracle.E_DUP_TS
    ok, _ = util.tables_equal(tabs, t)
    assert ok


def test_invalid_transactions_are_noops():
    tabs, types, bulk = util.small_bank(12, 40, n_branch=2, tpb=2, apt=3)
    bulk.params[0, 3] = 10_000          # account out of range
    bulk.params[2, 5] = -1              # branch out of range
    bulk.type[9] = 5                    # unregistered type
    out, st, res = _run(tabs, types, bulk, 3)
    assert st[3] == st[5] == st[9] == oracle.INVALID and (res[[3, 5, 9]] == 0).all()
    keep = np.setdiff1d(np.arange(40), [3, 5, 9])
    sub = wl.Bulk(bulk.type[keep], bulk.params[:, keep], bulk.ts[keep])
    out2, st2, res2 = _run(tabs, types, sub, 3)
    ok, msg = util.tables_equal(out, out2)
    assert ok, msg
    assert np.array_equal(res[keep], res2)


def test_capacity_error():
    tabs, types, bulk = util.small_bank(13, 30)
    tabs["history"] = wl.Table("history", ["i64"] * 5, [np.zeros(10, np.int64) for _ in range(5)],
                               0, 10, append=True)
    t = util.copy_tables(tabs)
    rc, _, _ = oracle.run_serial(t, types, bulk.type, bulk.params, bulk.ts, 3)
    assert rc == oracle.E_CAPACITY and t["history"].n_rows == 0


# ---------------------------------------------------------------------------
# generators

def test_generators_deterministic_and_skewed():
    a = wl.config3(n=2000, n_wh=2, items_per_w=1000, c_per_d=30).bulks[0]
    b = wl.config3(n=2000, n_wh=2, items_per_w=1000, c_per_d=30).bulks[0]
    assert np.array_equal(a.params, b.params) and np.array_equal(a.type, b.type)
    rng = np.random.default_rng(0)
    ids = wl.zipf_ids(rng, 640_000, 0.8, 200_000)
    share = (ids < 10_000).mean()        # hottest branch of 64 at 10k accounts each
    assert 0.38 < share < 0.45


# ---------------------------------------------------------------------------
# a transaction type that is not two-phase (Appendix D)

def test_rollback_new_order_has_no_effect():
    """A new-order that names the unused item id rolls back: stock, orders
    and order lines are as if it never ran, its status is ABORT and its
    results 0; the others run as plain new-orders (checked against the same
    bulk with the rolling-back transactions removed)."""
    tabs, types, bulk = util.small_order(41, 400, n_wh=2, d_per_w=3, c_per_d=4, items_per_w=50,
                                         rollback_frac=0.3)
    ipw = 50
    no = bulk.type == 1
    k = bulk.params[3]
    rb = no & np.array([(bulk.params[4:4 + 15, i][:k[i]] == ipw).any() for i in range(bulk.n)])
    assert 10 < int(rb.sum()) < int(no.sum())
    t_rb, st, res = _run(tabs, types, bulk, 16)
    assert (st[rb] == 1).all() and (res[rb] == 0).all()
    keep = ~rb
    plain = wl.Bulk(bulk.type[keep], bulk.params[:, keep], bulk.ts[keep])
    t_pl, st2, res2 = _run(tabs, wl.order_types(), plain, 16)
    assert np.array_equal(st[keep], st2) and np.array_equal(res[keep], res2)
    ok, msg = util.tables_equal(t_pl, t_rb)
    assert ok, msg
    # the Python twin agrees
    t_py = util.copy_tables(tabs)
    st3, res3 = ref.py_execute(t_py, types, bulk.type, bulk.params, bulk.ts, 16)
    assert np.array_equal(st3, st) and np.array_equal(res3, res)


def test_rollback_new_order_operations_skip_the_unused_item():
    tabs, types, bulk = util.small_order(42, 60, n_wh=1, d_per_w=2, c_per_d=2, items_per_w=20,
                                         rollback_frac=1.0)
    per = ref.bulk_ops(types, bulk.type, bulk.params, bulk.ts, util.sizes_of(tabs), util.roots_of(tabs))
    for i, _, ops in per:
        if bulk.type[i] == 1:
            assert len(ops) == bulk.params[3][i] - 1   # k items, one of them unused
            assert all(tab == "stock" and row < 20 for (tab, row) in ops)
