"""The no-allocation entry point: same results as gputx_execute_bulk.

gputx_execute_bulk_noalloc keeps its workspace in a static device array.
Two engines start from the same tables; one runs bulks through the
caller-workspace entry point, the other through the static one, two calls in
a row (the second bulk smaller, so stale contents of the array from the
first call are present).  Outputs, tables and appended rows must agree
exactly (integer work), and both agree with the oracle.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1103_3105_amd import workloads as wl
from tests import util

pytestmark = pytest.mark.gpu


def _tables_of(eng, tabs):
    out = util.copy_tables(tabs)
    for name, t in out.items():
        host = eng.table_host(name)
        for c in range(len(t.cols)):
            t.cols[c][:] = host[c]
        if t.append:
            t.n_rows = eng.row_count(name)
    return out


@pytest.mark.parametrize("strategy", ["AUTO", "TPL", "PART", "KSET"])
def test_noalloc_matches_workspace_entry_point(strategy):
    import torch
    from paper_1103_3105_amd import gputx
    rng = np.random.default_rng(401)
    n1, n2 = 40_000, 9_000
    tabs = wl.bank_tables(rng, 8, 80, 24_000, history_capacity=n1 + n2)
    b1 = wl.bank_bulk(rng, n1, 8, 80, 24_000, 0.8)
    b2 = wl.bank_bulk(rng, n2, 8, 80, 24_000, 0.0, ts0=n1)
    types = wl.bank_types()
    e_ws = gputx.Engine(tabs, types)
    e_na = gputx.Engine(tabs, types)
    o_tabs = util.copy_tables(tabs)
    try:
        for b in (b1, b2):
            rc, o_st, o_res = oracle.run_serial(o_tabs, types, b.type, b.params, b.ts, 3)
            assert rc == 0
            st1, res1, s1 = e_ws.execute(e_ws.bulk_to_device(b), gputx.STRATEGY[strategy], 3, ts_sorted=True)
            st2, res2, s2 = e_na.execute_noalloc(e_na.bulk_to_device(b), gputx.STRATEGY[strategy], 3,
                                                 ts_sorted=True)
            torch.cuda.synchronize()
            g1, g2 = gputx.stats_from(s1), gputx.stats_from(s2)
            assert g1.error == 0 and g2.error == 0, (g1.as_dict(), g2.as_dict())
            assert g1.as_dict() == g2.as_dict()
            assert np.array_equal(st1.cpu().numpy(), st2.cpu().numpy())
            assert np.array_equal(res1.cpu().numpy(), res2.cpu().numpy())
            assert np.array_equal(st2.cpu().numpy()[:b.n], o_st)
            assert np.array_equal(res2.cpu().numpy()[:b.n], o_res)
            t1, t2 = _tables_of(e_ws, tabs), _tables_of(e_na, tabs)
            ok, msg = util.tables_equal(t1, t2)
            assert ok, msg
            ok, msg = util.tables_equal(o_tabs, t2)
            assert ok, msg
    finally:
        e_ws.close()
        e_na.close()


def test_noalloc_rejects_bulks_beyond_the_static_workspace():
    import torch
    from paper_1103_3105_amd import gputx
    rng = np.random.default_rng(402)
    n = 1 << 20   # needs far more than 64 MiB of workspace
    tabs = wl.bank_tables(rng, 8, 80, 24_000, history_capacity=n)
    bulk = wl.bank_bulk(rng, n, 8, 80, 24_000, 0.0)
    eng = gputx.Engine(tabs, wl.bank_types())
    try:
        assert gputx.gputx_workspace_size(eng.h, n) > gputx.SCRATCH_BYTES
        with pytest.raises(gputx.GputxError) as ei:
            eng.execute_noalloc(eng.bulk_to_device(bulk), gputx.AUTO, 3, ts_sorted=True)
        assert ei.value.code == gputx.E_CAPACITY
        torch.cuda.synchronize()
        assert eng.row_count("history") == 0   # nothing ran
    finally:
        eng.close()
