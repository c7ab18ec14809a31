"""K-SET over a standing pool (Section 5.3's incremental k-set) against the
oracle: bulks added in timestamp order, interleaved with steps that each run
the pool's 0-set, give exactly the serial result over all bulks in order."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from oracle import reference as ref
from paper_1103_3105_amd import workloads as wl
from tests import util

pytestmark = pytest.mark.gpu


def _drain(pool, limit=1_000_000):
    for _ in range(limit):
        st = pool.state()
        assert st.error == 0, st.as_dict()
        if st.done_prefix == st.added:
            return st
        pool.step(8)
    raise AssertionError("pool did not drain")


def _run_pool(tabs, types, bulks, width, steps_between, max_ops=0, shuffle=False, **opts):
    import torch
    from paper_1103_3105_amd import gputx
    eng = gputx.Engine(tabs, types, **opts)
    try:
        total = sum(b.n for b in bulks)
        pool = gputx.Pool(eng, total, bulks[0].params.shape[0], width, max_ops=max_ops,
                          max_add=max(b.n for b in bulks))
        try:
            for k, b in enumerate(bulks):
                bb = wl.shuffled(b, np.random.default_rng(k)) if shuffle else b
                pool.add(eng.bulk_to_device(bb), ts_sorted=not shuffle)
                if steps_between[k % len(steps_between)]:
                    pool.step(steps_between[k % len(steps_between)])
            st = _drain(pool)
            g_st, g_res = pool.results(total)
            order = np.concatenate([np.argsort(b.ts, kind="stable") if shuffle else np.arange(b.n)
                                    for b in bulks])
        finally:
            pool.close()
        torch.cuda.synchronize()
        g_tabs = util.copy_tables(tabs)
        for name, t in g_tabs.items():
            host = eng.table_host(name)
            for c in range(len(t.cols)):
                t.cols[c][:] = host[c]
            if t.append:
                t.n_rows = eng.row_count(name)
    finally:
        eng.close()
    return st, g_tabs, g_st, g_res


def _oracle(tabs, types, bulks, width):
    o_tabs = util.copy_tables(tabs)
    outs = oracle.run_sequence(o_tabs, types, [(b, width) for b in bulks])
    return o_tabs, np.concatenate([s for s, _ in outs]), np.concatenate([r for _, r in outs])


def _check(tabs, types, bulks, width, got):
    st, g_tabs, g_st, g_res = got
    o_tabs, o_st, o_res = _oracle(tabs, types, bulks, width)
    assert np.array_equal(g_st, o_st), np.flatnonzero(g_st != o_st)[:8]
    assert np.array_equal(g_res, o_res)
    ok, msg = util.tables_equal(o_tabs, g_tabs)
    assert ok, msg
    assert st.committed == int((o_st == 0).sum()) and st.aborted == int((o_st == 1).sum())
    assert st.invalid == int((o_st == 2).sum())


def _bank_bulks(seed, sizes, theta, n_branch=8, tpb=10, apt=300):
    rng = np.random.default_rng(seed)
    nt, na = n_branch * tpb, n_branch * tpb * apt
    tabs = wl.bank_tables(rng, n_branch, nt, na, history_capacity=sum(sizes))
    bulks, ts0 = [], 0
    for m in sizes:
        bulks.append(wl.bank_bulk(rng, m, n_branch, nt, na, theta, ts0=ts0))
        ts0 += m + 7
    return tabs, bulks


@pytest.mark.parametrize("steps", [(0,), (1,), (3, 0, 1), (50,)])
def test_pool_bank_matches_serial(steps):
    tabs, bulks = _bank_bulks(81, [3000, 1, 4096, 777, 2500], 0.8)
    print("pool bank", steps, file=sys.stderr, flush=True)
    got = _run_pool(tabs, wl.bank_types(), bulks, 3, steps)
    _check(tabs, wl.bank_types(), bulks, 3, got)


def test_pool_subscriber_with_aborts_and_shuffled_input():
    rng = np.random.default_rng(82)
    tabs = wl.sub_tables(rng, 1500, occupancy=0.5)
    bulks, ts0 = [], 0
    for m in (2000, 3000, 500, 2500):
        b = wl.sub_bulk(rng, m, 1500, 0.9)
        bulks.append(wl.Bulk(b.type, b.params, np.arange(ts0, ts0 + m, dtype=np.int64)))
        ts0 += m
    got = _run_pool(tabs, wl.sub_types(), bulks, 14, (2, 0), shuffle=True, part_size=16)
    assert got[0].aborted > 0
    _check(tabs, wl.sub_types(), bulks, 14, got)


@pytest.mark.parametrize("rollback", [0.0, 0.1])
def test_pool_order_entry(rollback):
    rng = np.random.default_rng(83)
    bulks, ts0 = [], 0
    for m in (1500, 2500, 1000):
        b = wl.order_bulk(rng, m, 2, 10, 30, 300, rollback_frac=rollback)
        bulks.append(wl.Bulk(b.type, b.params, np.arange(ts0, ts0 + m, dtype=np.int64)))
        ts0 += m
    n_no = sum(int((b.type == 1).sum()) for b in bulks)
    n_l = sum(int(b.params[3][b.type == 1].sum()) for b in bulks)
    tabs = wl.order_tables(rng, 2, 10, 30, 300, n_no, n_l)
    types = wl.order_types(rollback=rollback > 0)
    got = _run_pool(tabs, types, bulks, 16, (1, 4))
    _check(tabs, types, bulks, 16, got)


def test_pool_waves_are_the_k_sets():
    """One bulk, drained one step at a time: each step runs exactly one k-set
    (the pool's 0-set), so the steps that ran something equal the depth + 1
    and each step's width is the size of that k-set."""
    import torch
    from paper_1103_3105_amd import gputx
    tabs, bulks = _bank_bulks(84, [3000], 0.8, n_branch=4, tpb=5, apt=20)
    b = bulks[0]
    per = ref.bulk_ops(wl.bank_types(), b.type, b.params, b.ts, util.sizes_of(tabs), util.roots_of(tabs))
    levels = ref.kahn_levels([o for _, _, o in per])
    eng = gputx.Engine(tabs, wl.bank_types())
    try:
        pool = gputx.Pool(eng, b.n, 4, 3, max_add=b.n)
        pool.add(eng.bulk_to_device(b), ts_sorted=True)
        widths = []
        while True:
            pool.step(1)
            st = pool.state()
            if st.last_width == 0:
                break
            widths.append(st.last_width)
        assert widths == [len(l) for l in levels]
        assert st.waves == len(levels) and st.done_prefix == b.n
        pool.close()
        torch.cuda.synchronize()
    finally:
        eng.close()


def test_pool_errors():
    """A bulk beyond the free slots is refused on the host with nothing
    added; a bulk whose ids do not follow the pool's is a bulk error, after
    which the pool runs nothing."""
    from paper_1103_3105_amd import gputx
    tabs, bulks = _bank_bulks(85, [500, 500], 0.0)
    eng = gputx.Engine(tabs, wl.bank_types())
    try:
        pool = gputx.Pool(eng, 512, 4, 3, max_add=600)
        pool.add(eng.bulk_to_device(bulks[0]), ts_sorted=True)
        with pytest.raises(gputx.GputxError) as ei:
            pool.add(eng.bulk_to_device(bulks[1]), ts_sorted=True)
        assert ei.value.code == gputx.E_CAPACITY
        st = _drain(pool)
        assert st.added == 500 and st.committed == 500
        pool.results(500)                 # frees the slots
        pool.add(eng.bulk_to_device(bulks[0]), ts_sorted=True)   # the same ids again
        pool.step(4)
        st = pool.state()
        assert st.error == gputx.E_UNSORTED and st.added == 500
        pool.close()
    finally:
        eng.close()
