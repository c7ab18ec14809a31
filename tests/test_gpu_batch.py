"""Batched form (many bulks, one HIP graph launch) against the serial oracle.

The graph is replayed several times with eager work and synchronisation in
between; every replay must equal the oracle's serial replay of the same job
sequence, and so must the plain one-bulk-per-launch form."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_1103_3105_amd import batching
from tests import util

pytestmark = pytest.mark.gpu


def _small(repeats):
    return batching.config4(n_bulks=24, lo=64, hi=8192, repeats=repeats, bank_branches=8,
                            accounts_per_branch=1000, n_wh=4, items_per_w=1000, c_per_d=30)


def _device_tables(eng, bw):
    out = util.copy_tables(bw.tables)
    for name, t in out.items():
        host = eng.table_host(name)
        for c in range(len(t.cols)):
            t.cols[c][:] = host[c]
        if t.append:
            t.n_rows = eng.row_count(name)
    return out


@pytest.mark.parametrize("strategy", ["AUTO", "KSET", "TPL", "PART"])
def test_batch_graph_replays_match_oracle(strategy):
    import torch
    from paper_1103_3105_amd import gputx
    replays = 3
    bw = _small(replays)
    print("batch", strategy, len(bw.jobs), bw.n_txns, file=sys.stderr, flush=True)
    eng = gputx.Engine(bw.tables, bw.types)
    o_tabs = util.copy_tables(bw.tables)
    try:
        jobs = batching.device_jobs(eng, bw, gputx.STRATEGY[strategy])
        batch = eng.batch(jobs)
        for r in range(replays):
            batch.launch()
            torch.cuda.synchronize()
            # eager work between replays
            _ = (jobs[0]["dev"]["params"] * 1).sum().item()
            want = oracle.run_sequence(o_tabs, bw.types, batching.sequence(bw), times=1)
            for k, (db, b) in enumerate(bw.jobs):
                s = batch.stats(k)
                assert s.error == 0, (r, k, s.as_dict())
                st = batch.outputs[k]["status"].cpu().numpy()[:b.n]
                res = batch.outputs[k]["results"].cpu().numpy()[:b.n]
                assert np.array_equal(st, want[k][0]), (r, k)
                assert np.array_equal(res, want[k][1]), (r, k)
            ok, msg = util.tables_equal(o_tabs, _device_tables(eng, bw))
            assert ok, (r, msg)
        batch.close()
    finally:
        eng.close()


def test_plain_form_matches_batched():
    import torch
    from paper_1103_3105_amd import gputx
    bw = _small(1)
    eng = gputx.Engine(bw.tables, bw.types)
    try:
        jobs = batching.device_jobs(eng, bw, gputx.AUTO)
        outs = [dict(status=torch.empty(max(b.n, 1), dtype=torch.int32, device=eng.device),
                     results=torch.empty((max(b.n, 1), batching.WIDTH[db]), dtype=torch.int64,
                                         device=eng.device),
                     stats=torch.empty(gputx.STATS_BYTES, dtype=torch.uint8, device=eng.device))
                for db, b in bw.jobs]
        lat = batching.run_plain(eng, jobs, outs)
        assert lat.shape[0] == len(jobs)
        o_tabs = util.copy_tables(bw.tables)
        want = oracle.run_sequence(o_tabs, bw.types, batching.sequence(bw))
        for k, (db, b) in enumerate(bw.jobs):
            assert np.array_equal(outs[k]["status"].cpu().numpy()[:b.n], want[k][0])
            assert np.array_equal(outs[k]["results"].cpu().numpy()[:b.n], want[k][1])
        ok, msg = util.tables_equal(o_tabs, _device_tables(eng, bw))
        assert ok, msg
    finally:
        eng.close()
