"""Benchmark: committed transactions per second of bulk execution on one MI355X.

Default workload: the scaled debit-credit bank -- 64 branches, 640 tellers,
6.4M accounts (int64 columns) -- and one bulk of 2^20 debit-credits with
uniform account keys, executed with ``gputx_execute_bulk`` (strategy chosen
by Algorithm 1 unless ``--strategy`` is given).  A step is one bulk through
the whole path: timestamp check, validation and scans, basic-operation
emission, the item-key radix sort, the ranking scan, features and strategy
choice, the executor and the batched append.  The bulk's arrays are already
resident in HBM when the timed region starts; the PCIe-inclusive rate (bulk
H2D + status/results D2H) is reported separately.

Prints one JSON line (see the ``out`` dict at the bottom).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "committed txns/sec on 1 MI355X, batched vs plain bulk; p50/p99 commit latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(args):
    from paper_1103_3105_amd import workloads as wl
    # append capacity for every bulk this run executes (timed, PCIe, strategy comparison)
    steps_total = args.warmup + 2 * args.steps + 24
    if args.workload == "bank":
        w = wl.config2(n=args.n, theta=args.theta, history_capacity=args.n * steps_total)
        name = (f"debit-credit bank: 64 branches, 640 tellers, 6.4M accounts; one bulk of "
                f"{args.n} txns, account Zipf theta={args.theta}")
        width = 3
    elif args.workload == "order":
        w = wl.config3(n=args.n)
        for t in ("orders", "order_line"):
            tab = w.tables[t]
            cap = tab.capacity * steps_total
            w.tables[t] = wl.Table(tab.name, tab.dtypes, [np.zeros(cap, np.int64) for _ in tab.cols],
                                   0, cap, append=True)
        name = f"order-entry: 16 warehouses, mix 45/43/12; one bulk of {args.n} txns"
        width = 16
    elif args.workload == "sub":
        w = wl.config5(n=args.n, n_sub=args.n_sub, theta=0.8)
        name = (f"subscriber: {args.n_sub} subscribers, 12 call-forwarding slots each, 80% reads; "
                f"one bulk of {args.n} txns, sid Zipf 0.8")
        width = 14
    else:
        raise SystemExit(f"unknown workload {args.workload}")
    return w, name, width


def phase_bytes(workload: str, n: int, m: int, key_passes: int, committed: int):
    """Algorithmic HBM bytes per phase of one bulk (what the method must move)."""
    exec_per_txn = {"bank": 32 + 8 + 4 + 24 + 40 + 3 * 16,
                    "order": 8 * 8 + 8 + 4 + 8 * 4 + 40 + 10 * 8,
                    "sub": 16 + 8 + 4 + 14 * 4 + 64}[workload]
    return {
        "order": 8 * n,
        "prepare": n * (32 + 4 + 4 + 8 + 8) + 2 * 2 * 8 * n,
        "emit": n * (32 + 8 + 8) + m * 12,
        "op_sort": m * (4 + 16 * key_passes),
        "rank": m * 44,
        "features": n * 8,
        "part": committed * exec_per_txn,
        "tpl": committed * exec_per_txn,
        "kset": committed * exec_per_txn,
    }


def oracle_baseline(w, bulk, width, budget_s=12.0):
    """The serial oracle on this host, on the same bulk from the same tables."""
    import oracle
    reps, elapsed, committed = 0, 0.0, 0
    while elapsed < budget_s and reps < 50:
        tabs = w.copy_tables()
        t0 = time.perf_counter()
        rc, st, _ = oracle.run_serial(tabs, w.types, bulk.type, bulk.params, bulk.ts, width)
        elapsed += time.perf_counter() - t0
        assert rc == 0
        committed += int((st == 0).sum())
        reps += 1
    return {"value": committed / elapsed, "unit": "txn/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} serial runs of the same {bulk.n}-txn bulk ({elapsed:.1f} s)"}


def bench_batch(args):
    """Config-4 form: 512 uneven bulks over two databases, batched (one graph
    launch) vs plain (one execute + wait per bulk)."""
    import torch
    import oracle  # noqa: F401
    from paper_1103_3105_amd import batching, gputx
    reps = args.warmup + args.steps + 2
    log(f"[bench] generating the 512-bulk batch workload")
    bw = batching.config4(n_bulks=args.bulks, repeats=reps)
    n_txn = bw.n_txns
    eng = gputx.Engine(bw.tables, bw.types)
    jobs = batching.device_jobs(eng, bw, gputx.STRATEGY[args.strategy])
    o_tabs = {k: v.copy() for k, v in bw.tables.items()}
    # plain form once, with parity against the oracle
    gputx.gputx_phase_timing(eng.h, True)
    outs = [dict(status=torch.empty(max(b.n, 1), dtype=torch.int32, device=eng.device),
                 results=torch.empty((max(b.n, 1), batching.WIDTH[db]), dtype=torch.int64,
                                     device=eng.device),
                 stats=torch.empty(gputx.STATS_BYTES, dtype=torch.uint8, device=eng.device))
            for db, b in bw.jobs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat = batching.run_plain(eng, jobs, outs)
    plain_s = time.perf_counter() - t0
    phases, nb = gputx.gputx_phase_times(eng.h)
    gputx.gputx_phase_timing(eng.h, False)
    want = batching.oracle_replay(bw, o_tabs)
    parity = all(np.array_equal(outs[k]["status"].cpu().numpy()[:b.n], want[k][0]) and
                 np.array_equal(outs[k]["results"].cpu().numpy()[:b.n], want[k][1])
                 for k, (db, b) in enumerate(bw.jobs))
    committed_plain = sum(gputx.stats_from(o["stats"]).committed for o in outs)
    log(f"[bench] plain: {plain_s:.3f} s, parity={parity}")
    batch = eng.batch(jobs)
    for _ in range(args.warmup):
        batch.launch()
    torch.cuda.synchronize()
    # parity of the batched form on its first timed replay (outside timing)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record()
    for k in range(args.steps):
        batch.launch()
        ev[k + 1].record()
    torch.cuda.synchronize()
    per = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)])
    committed = sum(batch.stats(k).committed for k in range(len(bw.jobs)))
    errors = sum(batch.stats(k).error != 0 for k in range(len(bw.jobs)))
    batched_value = committed * args.steps / (per.sum() / 1e3)
    plain_value = committed_plain / plain_s
    log(f"[bench] batched: {per.mean():.1f} ms/launch, {batched_value / 1e6:.2f}M txn/s; "
        f"plain {plain_value / 1e6:.2f}M txn/s")
    return dict(batched_value=batched_value, plain_value=plain_value, n_txns=n_txn,
                n_bulks=len(bw.jobs), parity=bool(parity) and errors == 0,
                ms_per_launch=float(per.mean()),
                plain_bulk_latency_ms={"p50": float(np.percentile(lat, 50) * 1e3),
                                       "p99": float(np.percentile(lat, 99) * 1e3)},
                phases_ms_total_plain={k: round(v, 3) for k, v in phases.items()})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="bank", choices=["bank", "order", "sub"])
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--n-sub", type=int, default=10_000_000)
    ap.add_argument("--theta", type=float, default=0.0)
    ap.add_argument("--strategy", default="AUTO", choices=["AUTO", "TPL", "PART", "KSET"])
    ap.add_argument("--compare", action="store_true", help="also time every strategy")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--batch-only", action="store_true", help="only the 512-bulk batched form")
    ap.add_argument("--bulks", type=int, default=512)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(DESIGN.md describes how it would shard)", file=sys.stderr)
        raise SystemExit(2)

    import torch
    import oracle
    from paper_1103_3105_amd import gputx

    if args.batch_only:
        print(json.dumps(bench_batch(args)), flush=True)
        return

    log(f"[bench] generating {args.workload} n={args.n}")
    w, wname, width = make_workload(args)
    bulk = w.bulks[0]
    eng = gputx.Engine(w.tables, w.types, part_size=(128 if args.workload == "sub" else 1))
    dev = eng.bulk_to_device(bulk)
    n = bulk.n
    status = torch.empty(n, dtype=torch.int32, device=eng.device)
    results = torch.empty((n, width), dtype=torch.int64, device=eng.device)
    stats = torch.empty(gputx.STATS_BYTES, dtype=torch.uint8, device=eng.device)
    stream = torch.cuda.current_stream()

    def step(strategy):
        eng.execute(dev, gputx.STRATEGY[strategy], width, ts_sorted=True, status=status,
                    results=results, stats=stats, stream=stream)

    # parity on the first warm-up bulk (outside timing)
    log("[bench] parity check vs oracle on the first bulk")
    step(args.strategy)
    torch.cuda.synchronize()
    s0 = gputx.stats_from(stats)
    o_tabs = w.copy_tables()
    rc, o_st, o_res = oracle.run_serial(o_tabs, w.types, bulk.type, bulk.params, bulk.ts, width)
    parity = (rc == 0 and s0.error == 0 and np.array_equal(status.cpu().numpy(), o_st)
              and np.array_equal(results.cpu().numpy(), o_res))
    for name, t in o_tabs.items():
        if t.append:
            continue
        host = eng.table_host(name)
        parity = parity and all(np.array_equal(h, c) for h, c in zip(host, t.cols))
    log(f"[bench] parity={parity} stats={s0.as_dict()}")

    for _ in range(max(args.warmup - 1, 0)):
        step(args.strategy)
    torch.cuda.synchronize()

    gputx.gputx_phase_timing(eng.h, True)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(stream)
    for k in range(args.steps):
        step(args.strategy)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_step = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)])
    total_ms = float(evs[0].elapsed_time(evs[-1]))
    phases, nb = gputx.gputx_phase_times(eng.h)
    gputx.gputx_phase_timing(eng.h, False)
    s = gputx.stats_from(stats)
    committed = s.committed
    value = committed * args.steps / (total_ms / 1e3)
    log(f"[bench] {args.steps} steps {total_ms:.2f} ms (wall {wall*1e3:.1f} ms) "
        f"strategy={gputx.STRATEGY_NAME[s.chosen]} waves={s.waves} depth={s.depth} w0={s.w0}")
    log("[bench] phases (ms/bulk): " + ", ".join(f"{k}={v / max(nb, 1):.3f}" for k, v in phases.items()))

    # roofline of the dominant phase (kernel group)
    pb = phase_bytes(args.workload, n, s.n_ops, key_passes(w.tables), committed)
    dom = max((k for k in phases if k in pb), key=lambda k: phases[k])
    dom_ms = phases[dom] / max(nb, 1)
    achieved = pb[dom] / (dom_ms / 1e3) / 1e9 if dom_ms > 0 else 0.0
    roofline = {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 6), "traffic": None, "kernel": dom,
                "bytes_per_launch": pb[dom], "ms_per_launch": round(dom_ms, 4)}

    # PCIe-inclusive rate: bulk H2D + status/results D2H around each bulk
    pin = {k: torch.empty_like(v, device="cpu").pin_memory() for k, v in dev.items()}
    for k in pin:
        pin[k].copy_(dev[k])
    st_h = torch.empty_like(status, device="cpu").pin_memory()
    res_h = torch.empty_like(results, device="cpu").pin_memory()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    reps = max(2, args.steps // 2)
    for _ in range(reps):
        for k in dev:
            dev[k].copy_(pin[k], non_blocking=True)
        step(args.strategy)
        st_h.copy_(status, non_blocking=True)
        res_h.copy_(results, non_blocking=True)
    e1.record(stream)
    torch.cuda.synchronize()
    pcie_value = committed * reps / (e0.elapsed_time(e1) / 1e3)

    extra = {}
    if args.compare:
        for strat in ("TPL", "PART", "KSET"):
            step(strat)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            reps = 3
            for _ in range(reps):
                step(strat)
            b.record(stream)
            torch.cuda.synchronize()
            sx = gputx.stats_from(stats)
            ms = a.elapsed_time(b) / reps
            extra[strat] = {"ms_per_bulk": round(ms, 3), "txn_per_s": round(sx.committed / (ms / 1e3)),
                            "error": sx.error}
            log(f"[bench] {strat}: {ms:.3f} ms/bulk")

    cpu = None
    if not args.no_cpu:
        log("[bench] timing the serial oracle on the host")
        cpu = oracle_baseline(w, bulk, width)

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "txn/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total_ms / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": wname, "form": "plain (one bulk per launch sequence)",
                   "bulk_txns": n, "strategy": gputx.STRATEGY_NAME[s.chosen],
                   "requested": args.strategy},
        "latency_ms": {"p50": round(float(np.percentile(per_step, 50)), 4),
                       "p99": round(float(np.percentile(per_step, 99)), 4)},
        "pcie_inclusive_value": round(pcie_value, 1),
        "parity_vs_oracle": bool(parity),
        "bulk_stats": {k: v for k, v in s.as_dict().items()},
        "phases_ms_per_bulk": {k: round(v / max(nb, 1), 4) for k, v in phases.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if extra:
        out["strategies"] = extra
    eng.close()
    print(json.dumps(out), flush=True)


def key_passes(tables) -> int:
    """8-bit digits of the item-key sort: keys span every non-append table's rows."""
    total = sum(t.n_rows for t in tables.values() if not t.append)
    return max(1, (int(total - 1).bit_length() + 7) // 8)


if __name__ == "__main__":
    main()
