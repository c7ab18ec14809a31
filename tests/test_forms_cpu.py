"""Host-side logic of the batched and served forms and of the calibration
(CPU only; the oracle stands in for the GPU where an executor is needed)."""
from __future__ import annotations

import numpy as np

import oracle
from paper_1103_3105_amd import autotune, batching, serving, workloads as wl
from tests import util


def test_config4_jobs_structure():
    bw = batching.config4(n_bulks=40, lo=64, hi=4096, bank_branches=4, accounts_per_branch=500,
                          n_wh=2, items_per_w=500, c_per_d=20)
    assert len(bw.jobs) == 40
    sizes = np.array([b.n for _, b in bw.jobs])
    assert sizes.min() >= 64 and sizes.max() <= 4096
    ts = np.concatenate([b.ts for _, b in bw.jobs])
    assert np.all(np.diff(ts) > 0)                    # globally increasing ids
    dbs = {db for db, _ in bw.jobs}
    assert dbs == {"bank", "order"}
    for db, b in bw.jobs:
        assert set(np.unique(b.type)) <= ({0} if db == "bank" else {1, 2, 3})
    # both databases' tables are present once, with room for every append
    hist = bw.tables["history"]
    assert hist.capacity >= sum(b.n for db, b in bw.jobs if db == "bank")


def test_batch_oracle_replay_is_per_database_serial_order():
    bw = batching.config4(n_bulks=12, lo=32, hi=512, repeats=1, bank_branches=2,
                          accounts_per_branch=100, n_wh=1, items_per_w=200, c_per_d=10)
    t1 = util.copy_tables(bw.tables)
    got = oracle.run_sequence(t1, bw.types, batching.sequence(bw))
    # the same as one serial run per database over the concatenated bulks
    t2 = util.copy_tables(bw.tables)
    for db, width in (("bank", 3), ("order", 16)):
        bulks = [b for d, b in bw.jobs if d == db]
        types = [t for t in bw.types if (t.type_id == 0) == (db == "bank")]
        cat = wl.Bulk(np.concatenate([b.type for b in bulks]),
                      np.concatenate([b.params for b in bulks], axis=1),
                      np.concatenate([b.ts for b in bulks]))
        rc, st, res = oracle.run_serial(t2, types, cat.type, cat.params, cat.ts, width)
        assert rc == 0
        mine = [k for k, (d, _) in enumerate(bw.jobs) if d == db]
        assert np.array_equal(np.concatenate([got[k][0] for k in mine]), st)
        assert np.array_equal(np.concatenate([got[k][1] for k in mine]), res)
    ok, msg = util.tables_equal(t1, t2)
    assert ok, msg


def test_trace_is_poisson_in_arrival_order():
    tr = serving.make_trace(2_000_000, 0.5, 10_000, seed=3)
    assert np.all(np.diff(tr.arrival_ns) >= 0) and np.all(np.diff(tr.ts) == 1)
    rate = tr.n / (tr.arrival_ns[-1] / 1e9)
    assert abs(rate / 2e6 - 1) < 0.01
    gaps = np.diff(tr.arrival_ns).astype(np.float64)
    assert abs(gaps.std() / gaps.mean() - 1) < 0.02   # exponential gaps: CV = 1
    assert set(np.unique(tr.type)) <= set(range(4, 10))


def test_fit_thresholds_recovers_the_rule():
    # K-SET is fastest for wide 0-sets, PART otherwise: the fit must separate them
    samples = []
    for w0 in (10, 100, 1000, 20000, 50000):
        fast = "KSET" if w0 >= 20000 else "PART"
        ms = {s: (1.0 if s == fast else 5.0) for s in autotune.STRATS}
        samples.append(autotune.Sample(w0=w0, depth=w0 // 10, cross=0, ms=ms))
    th = autotune.fit_thresholds(samples)
    for s in samples:
        pick = autotune.choose(s.w0, s.depth, s.cross, th["w0_bar"], th["c_bar"], th["d_bar"])
        assert s.ms[pick] == 1.0
    assert th["total_ms"] == len(samples)


def test_choose_matches_reference_rule():
    from oracle import reference as ref
    rng = np.random.default_rng(0)
    for _ in range(200):
        w0, d, c = (int(x) for x in rng.integers(0, 100, 3))
        wb, cb, db = (int(x) for x in rng.integers(0, 100, 3))
        want = ref.choose_strategy(w0, d, c, wb, cb, db)
        got = autotune.choose(w0, d, c, wb, cb, db)
        # the engine runs PART with cross-partition transactions under TPL (Section 5.2)
        assert got == ("TPL" if (want == "PART" and c > 0) else want)
