"""The paper's CPU counterpart (Section 6.3): the partitioned host executor
must equal the serial oracle exactly, and its routing must agree with the
partition sets of the Python reference (CPU only)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import reference as ref
from paper_1103_3105_amd import workloads as wl
from tests import util


def _cases():
    rng = np.random.default_rng(91)
    bank_t = wl.bank_tables(rng, 8, 80, 8000, history_capacity=6000)
    bank_b = wl.bank_bulk(rng, 6000, 8, 80, 8000, 0.8, remote_frac=0.1)
    o_t, o_ty, o_b = util.small_order(92, 4000, n_wh=4, d_per_w=5, c_per_d=20, items_per_w=200)
    s_t, s_ty, s_b = util.small_sub(93, 4000, n_sub=500)
    return {"bank": (bank_t, wl.bank_types(), bank_b, 3, 1),
            "order": (o_t, o_ty, o_b, 16, 1),
            "sub": (s_t, s_ty, s_b, 14, 16)}


@pytest.mark.parametrize("name", ["bank", "order", "sub"])
def test_partition_ids_match_reference(name):
    tabs, types, bulk, _, ps = _cases()[name]
    k = 600
    sub = wl.Bulk(bulk.type[:k], bulk.params[:, :k], bulk.ts[:k])
    got = oracle.partition_ids(tabs, types, sub.type, sub.params, ps)
    per = ref.bulk_ops(types, sub.type, sub.params, sub.ts, util.sizes_of(tabs), util.roots_of(tabs))
    for (i, _, ops) in per:
        parts = ref.partitions_of(ops, util.roots_of(tabs), ps)
        if not ops:
            continue   # invalid: never routed
        want = next(iter(parts)) if len(parts) == 1 else -1
        assert got[i] == want, (i, parts, got[i])
    if name == "bank":
        assert (got < 0).any()          # the remote tellers span two branches


@pytest.mark.parametrize("threads", [1, 3, 8])
@pytest.mark.parametrize("name", ["bank", "order", "sub"])
def test_partitioned_equals_serial(name, threads):
    tabs, types, bulk, width, ps = _cases()[name]
    if name != "bank":
        bulk = wl.shuffled(bulk, np.random.default_rng(4), gapped=True)
    a, b = util.copy_tables(tabs), util.copy_tables(tabs)
    rc1, st1, r1 = oracle.run_serial(a, types, bulk.type, bulk.params, bulk.ts, width)
    part = oracle.partition_ids(tabs, types, bulk.type, bulk.params, ps)
    rc2, st2, r2 = oracle.run_partitioned(b, types, bulk.type, bulk.params, bulk.ts, width, part,
                                          threads)
    assert rc1 == rc2 == 0
    assert np.array_equal(st1, st2) and np.array_equal(r1, r2)
    ok, msg = util.tables_equal(a, b)
    assert ok, msg


def test_partitioned_errors_leave_tables_untouched():
    tabs, types, bulk, width, ps = _cases()["bank"]
    part = oracle.partition_ids(tabs, types, bulk.type, bulk.params, ps)
    ts = bulk.ts.copy()
    ts[5] = ts[4]
    t = util.copy_tables(tabs)
    rc, _, _ = oracle.run_partitioned(t, types, bulk.type, bulk.params, ts, width, part, 4)
    assert rc == oracle.E_DUP_TS
    t2 = util.copy_tables(tabs)
    t2["history"].capacity = 10
    rc, _, _ = oracle.run_partitioned(t2, types, bulk.type, bulk.params, bulk.ts, width, part, 4)
    assert rc == oracle.E_CAPACITY
    for k in tabs:
        for c0, c1 in zip(tabs[k].cols, t[k].cols):
            assert np.array_equal(c0, c1)
