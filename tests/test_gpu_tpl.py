"""Counter-based TPL: deterministic results under repeated contended runs,
and the bounded-wait path (a tiny spin limit set from the host makes a long
lock wait expire; the bulk reports GPUTX_E_DEADLOCK and every wave exits)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_1103_3105_amd import workloads as wl
from tests import util

pytestmark = pytest.mark.gpu


def test_tpl_deterministic_under_repeats():
    import torch
    from paper_1103_3105_amd import gputx
    tabs, types, bulk = util.small_bank(41, 30_000, n_branch=4, tpb=5, apt=50, theta=0.8)
    o_tabs = util.copy_tables(tabs)
    rc, o_st, o_res = oracle.run_serial(o_tabs, types, bulk.type, bulk.params, bulk.ts, 3)
    assert rc == 0
    eng = gputx.Engine(tabs, types)
    try:
        dev = eng.bulk_to_device(bulk)
        snap = {k: [c.clone() for c in eng.cols[k]] for k in ("account", "teller", "branch")}
        for rep in range(30):
            for k, cols in snap.items():           # restore the tables between runs
                for dst, src in zip(eng.cols[k], cols):
                    dst.copy_(src)
            eng.truncate_appends()
            st, res, stats = eng.execute(dev, gputx.TPL, 3, ts_sorted=True)
            torch.cuda.synchronize()
            s = gputx.stats_from(stats)
            assert s.error == 0 and s.chosen == gputx.TPL, (rep, s.as_dict())
            assert np.array_equal(st.cpu().numpy(), o_st), rep
            assert np.array_equal(res.cpu().numpy(), o_res), rep
            for k in snap:
                assert np.array_equal(eng.table_host(k)[0], o_tabs[k].cols[0]), (rep, k)
    finally:
        eng.close()


def test_bounded_wait_reports_deadlock_and_drains():
    import torch
    from paper_1103_3105_amd import gputx
    w = wl.config1()   # one 4096-long dependency chain: late lanes wait for milliseconds
    eng = gputx.Engine(w.tables, w.types, spin_limit_ms=1)
    try:
        dev = eng.bulk_to_device(w.bulks[0])
        st, res, stats = eng.execute(dev, gputx.TPL, 3, ts_sorted=True)
        torch.cuda.synchronize()
        s = gputx.stats_from(stats)
        print("watchdog", s.as_dict(), file=sys.stderr, flush=True)
        assert s.error == gputx.E_DEADLOCK
        # the engine stays usable: a normal limit runs a fresh bulk to completion
        eng.set_options(spin_limit_ms=5000)
        eng.truncate_appends()
        st, res, stats = eng.execute(dev, gputx.PART, 3, ts_sorted=True)
        torch.cuda.synchronize()
        assert gputx.stats_from(stats).error == 0
    finally:
        eng.close()
