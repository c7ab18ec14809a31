"""Seeded synthetic workloads for bulk transaction execution.

This module only draws data: initial tables, transaction signatures
<id, type, params> (Section 3.2) and arrival traces.  It holds none of the
method's arithmetic (no procedure semantics, no dependency analysis), so the
serial oracle and the GPU engine can both consume its arrays.

The paper evaluates on TPC-B, TPC-C and TM-1 (Section 6.1, Appendix E); their
kits are not available, so each workload below is a synthetic stand-in with
the shape the paper describes: a tree-shaped debit-credit bank (one type,
branch as partition key), a mixed order-entry schema (three types, warehouse
as partition key) and a subscriber / call-forwarding schema (six types,
subscriber id as partition key, 80% read-only).

Layouts
-------
* A table is column-major: one numpy array per fixed-length column
  (Appendix E, column-based store).  Append-only tables are allocated at
  their capacity; rows past ``n_rows`` are zero.
* A bulk is structure-of-arrays: ``type[n] int32``, ``params[P][n] int64``
  (param-major so that one parameter of consecutive transactions is
  contiguous) and ``ts[n] int64`` (the transaction id used as timestamp).
"""
from __future__ import annotations

import dataclasses
import functools
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

# Procedure names.  Each side (oracle, engine) maps these names to its own
# procedure enumeration.
PROCS = (
    "DEBIT_CREDIT",
    "NEW_ORDER",
    "PAYMENT",
    "ORDER_STATUS",
    "GET_SUB",
    "GET_CF",
    "UPD_SUB_FIELD",
    "UPD_LOC",
    "INS_CF",
    "DEL_CF",
    "NEW_ORDER_RB",
)

# Role lists: the tables a procedure is bound to, in order.
BANK_ROLES = ("account", "teller", "branch", "history")
ORDER_ROLES = ("warehouse", "district", "customer", "stock", "orders", "order_line")
SUB_ROLES = ("subscriber", "call_fwd")

NO_MAX_ITEMS = 15          # new-order lines per transaction, upper bound
NO_PARAMS = 4 + 2 * NO_MAX_ITEMS   # w, d, c, k, item[15], q[15]
CF_SLOTS = 12              # call-forwarding slots per subscriber: 4 types x 3 starts
SUB_FIELDS = 4             # int32 bit/byte fields of a subscriber
SUB_LOCS = 10              # int32 location fields of a subscriber


@dataclasses.dataclass
class Table:
    name: str
    dtypes: List[str]              # "i64" | "i32" per column
    cols: List[np.ndarray]         # each of length ``capacity``
    n_rows: int
    capacity: int
    append: bool = False
    root: Optional[str] = None     # table holding the partition root key
    root_div: int = 0              # rows of this table per root key (0: none)

    def copy(self) -> "Table":
        return dataclasses.replace(self, cols=[c.copy() for c in self.cols])


@dataclasses.dataclass
class TypeDesc:
    type_id: int
    proc: str
    n_params: int
    n_results: int
    tables: Sequence[str]
    root_key: bool = False         # lock only the partition root (Section 5.1)
    single_partition: bool = True  # DBA annotation (Appendix E)


@dataclasses.dataclass
class Bulk:
    type: np.ndarray    # int32 [n]
    params: np.ndarray  # int64 [P, n]
    ts: np.ndarray      # int64 [n]

    @property
    def n(self) -> int:
        return int(self.type.shape[0])


@dataclasses.dataclass
class Workload:
    name: str
    tables: Dict[str, Table]
    types: List[TypeDesc]
    bulks: List[Bulk]
    n_results: int
    meta: dict = dataclasses.field(default_factory=dict)

    def copy_tables(self) -> Dict[str, Table]:
        return {k: v.copy() for k, v in self.tables.items()}


# ---------------------------------------------------------------------------
# random helpers

def rng_for(cfg: int, stream: int = 0) -> np.random.Generator:
    """Independent PCG64 stream ``stream`` of workload ``cfg``."""
    ss = np.random.SeedSequence(1103_000 + cfg)
    return np.random.default_rng(ss.spawn(stream + 1)[stream])


def zipf_ids(rng: np.random.Generator, n_keys: int, theta: float, size: int) -> np.ndarray:
    """Draw ``size`` ids in [0, n_keys) with P(id = r-1) proportional to r^-theta.

    Exact inverse-CDF sampling over a float64 cumulative sum; theta = 0 is
    uniform.  Ids are unscrambled: id 0 is the hottest.
    """
    if theta == 0.0:
        return rng.integers(0, n_keys, size=size, dtype=np.int64)
    cdf = _zipf_cdf(n_keys, theta)
    u = rng.random(size)
    ids = np.searchsorted(cdf, u, side="right").astype(np.int64)
    return np.minimum(ids, n_keys - 1)


@functools.lru_cache(maxsize=8)
def _zipf_cdf(n_keys: int, theta: float) -> np.ndarray:
    w = np.arange(1, n_keys + 1, dtype=np.float64) ** (-theta)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    return cdf


def _col(n: int, dt: str) -> np.ndarray:
    return np.zeros(n, dtype=np.int64 if dt == "i64" else np.int32)


# ---------------------------------------------------------------------------
# debit-credit bank (TPC-B stand-in)

def bank_tables(rng: np.random.Generator, n_branch: int, n_teller: int, n_account: int,
                history_capacity: int) -> Dict[str, Table]:
    """Branch / teller / account balances (uniform 0..1e6) plus an empty history.

    Balance is column 0 of branch, teller and account; the remaining columns
    are the static keys of the schema.
    """
    tpb = n_teller // n_branch
    apt = n_account // n_teller
    acct_id = np.arange(n_account, dtype=np.int64)
    account = Table("account", ["i64"] * 4,
                    [rng.integers(0, 1_000_001, n_account, dtype=np.int64),
                     acct_id, acct_id // apt, acct_id // (apt * tpb)],
                    n_account, n_account, root="branch", root_div=apt * tpb)
    tel_id = np.arange(n_teller, dtype=np.int64)
    teller = Table("teller", ["i64"] * 3,
                   [rng.integers(0, 1_000_001, n_teller, dtype=np.int64), tel_id, tel_id // tpb],
                   n_teller, n_teller, root="branch", root_div=tpb)
    branch = Table("branch", ["i64"] * 2,
                   [rng.integers(0, 1_000_001, n_branch, dtype=np.int64),
                    np.arange(n_branch, dtype=np.int64)],
                   n_branch, n_branch, root="branch", root_div=1)
    history = Table("history", ["i64"] * 5, [_col(history_capacity, "i64") for _ in range(5)],
                    0, history_capacity, append=True)
    return {t.name: t for t in (account, teller, branch, history)}


def bank_bulk(rng: np.random.Generator, n: int, n_branch: int, n_teller: int, n_account: int,
              theta: float, ts0: int = 0, remote_frac: float = 0.0) -> Bulk:
    """n debit-credits: acct Zipf(theta), teller and branch of that account,
    delta uniform in [-99999, 99999], ts = ts0 .. ts0+n-1.

    With ``remote_frac`` > 0 (and more than one branch), that fraction of the
    transactions goes through a teller drawn uniformly from another branch
    (TPC-B's remote account holders): their account and their teller/branch
    rows then lie under different partition roots."""
    apt = n_account // n_teller
    tpb = n_teller // n_branch
    acct = zipf_ids(rng, n_account, theta, n)
    teller = acct // apt
    if remote_frac > 0 and n_branch > 1:
        remote = rng.random(n) < remote_frac
        k = int(remote.sum())
        home = teller[remote] // tpb
        other = (home + rng.integers(1, n_branch, k)) % n_branch
        teller = teller.copy()
        teller[remote] = other * tpb + rng.integers(0, tpb, k)
    branch = teller // tpb
    delta = rng.integers(-99_999, 100_000, n, dtype=np.int64)
    params = np.stack([acct, teller, branch, delta]).astype(np.int64)
    return Bulk(np.zeros(n, np.int32), np.ascontiguousarray(params),
                np.arange(ts0, ts0 + n, dtype=np.int64))


def bank_types(root_key: bool = False) -> List[TypeDesc]:
    return [TypeDesc(0, "DEBIT_CREDIT", 4, 3, BANK_ROLES, root_key=root_key)]


def config1(root_key: bool = False) -> Workload:
    """Tiny bank: 1 branch, 10 tellers, 1000 accounts, one bulk of 4096."""
    rng = rng_for(1)
    n = 4096
    tabs = bank_tables(rng, 1, 10, 1000, history_capacity=n)
    bulk = bank_bulk(rng, n, 1, 10, 1000, 0.0)
    return Workload("bank-tiny", tabs, bank_types(root_key), [bulk], 3,
                    meta=dict(n_branch=1, n_teller=10, n_account=1000))


def config2(n: int = 1 << 20, theta: float = 0.0, n_branch: int = 64,
            accounts_per_branch: int = 100_000, root_key: bool = False,
            history_capacity: Optional[int] = None) -> Workload:
    """Scaled bank: 64 branches, 640 tellers, 6.4M accounts; one bulk of n
    debit-credits with Zipf(theta) account keys."""
    th_idx = {0.0: 0, 0.8: 1, 0.99: 2}.get(theta, 3)
    rng_t = rng_for(2, 0)
    rng_b = rng_for(2, 1 + 8 * th_idx + int(round(math.log2(max(n, 1)))) % 8)
    n_teller = n_branch * 10
    n_account = n_branch * accounts_per_branch
    tabs = bank_tables(rng_t, n_branch, n_teller, n_account,
                       history_capacity=history_capacity or n)
    bulk = bank_bulk(rng_b, n, n_branch, n_teller, n_account, theta)
    return Workload(f"bank-{n_branch}b-n{n}-theta{theta}", tabs, bank_types(root_key), [bulk], 3,
                    meta=dict(n_branch=n_branch, n_teller=n_teller, n_account=n_account,
                              theta=theta))


# ---------------------------------------------------------------------------
# order-entry (TPC-C stand-in)

def order_tables(rng: np.random.Generator, n_wh: int, d_per_w: int, c_per_d: int,
                 items_per_w: int, orders_capacity: int, lines_capacity: int) -> Dict[str, Table]:
    """Warehouse / district / customer int64 balances (uniform 0..1e6),
    stock int32 quantities (uniform 10..100), empty orders and order_line."""
    n_d = n_wh * d_per_w
    n_c = n_d * c_per_d
    n_s = n_wh * items_per_w
    wh = Table("warehouse", ["i64"], [rng.integers(0, 1_000_001, n_wh, dtype=np.int64)],
               n_wh, n_wh, root="warehouse", root_div=1)
    di = Table("district", ["i64"], [rng.integers(0, 1_000_001, n_d, dtype=np.int64)],
               n_d, n_d, root="warehouse", root_div=d_per_w)
    cu = Table("customer", ["i64"], [rng.integers(0, 1_000_001, n_c, dtype=np.int64)],
               n_c, n_c, root="warehouse", root_div=d_per_w * c_per_d)
    st = Table("stock", ["i32"], [rng.integers(10, 101, n_s, dtype=np.int64).astype(np.int32)],
               n_s, n_s, root="warehouse", root_div=items_per_w)
    orders = Table("orders", ["i64"] * 5, [_col(orders_capacity, "i64") for _ in range(5)],
                   0, orders_capacity, append=True)
    lines = Table("order_line", ["i64"] * 5, [_col(lines_capacity, "i64") for _ in range(5)],
                  0, lines_capacity, append=True)
    return {t.name: t for t in (wh, di, cu, st, orders, lines)}


def order_types(root_key: bool = False, rollback: bool = False) -> List[TypeDesc]:
    """rollback: new-order registered as the procedure that is not two-phase
    (an unused item id makes it roll back its stock updates)."""
    return [
        TypeDesc(1, "NEW_ORDER_RB" if rollback else "NEW_ORDER", NO_PARAMS, 1 + NO_MAX_ITEMS,
                 ORDER_ROLES, root_key=root_key),
        TypeDesc(2, "PAYMENT", 4, 3, ORDER_ROLES, root_key=root_key),
        TypeDesc(3, "ORDER_STATUS", 3, 1, ORDER_ROLES, root_key=root_key),
    ]


def order_bulk(rng: np.random.Generator, n: int, n_wh: int, d_per_w: int, c_per_d: int,
               items_per_w: int, ts0: int = 0, mix=(0.45, 0.43, 0.12),
               rollback_frac: float = 0.0) -> Bulk:
    """Mixed bulk: new-order (k uniform 5..15 distinct items, q uniform 1..10),
    payment (h uniform 1..5000), order-status; w, d, c uniform.

    rollback_frac: that fraction of new-orders names the unused item id
    (items_per_w) as its last item, as TPC-C's 1% of new-orders that roll
    back (for new-order registered as NEW_ORDER_RB)."""
    kind = rng.choice(3, size=n, p=np.asarray(mix, dtype=np.float64))
    types = (kind + 1).astype(np.int32)
    params = np.zeros((NO_PARAMS, n), dtype=np.int64)
    params[0] = rng.integers(0, n_wh, n)
    params[1] = rng.integers(0, d_per_w, n)
    params[2] = rng.integers(0, c_per_d, n)
    no = np.nonzero(kind == 0)[0]
    k = np.minimum(rng.integers(5, NO_MAX_ITEMS + 1, no.size), items_per_w)
    live = np.arange(NO_MAX_ITEMS)[None, :] < k[:, None]
    items = rng.integers(0, items_per_w, (no.size, NO_MAX_ITEMS))
    # redraw rows with a repeated live item until each row's k items are distinct
    while True:
        tagged = np.where(live, items, -1 - np.arange(NO_MAX_ITEMS)[None, :])
        s = np.sort(tagged, axis=1)
        bad = np.nonzero((s[:, 1:] == s[:, :-1]).any(axis=1))[0]
        if bad.size == 0:
            break
        items[bad] = rng.integers(0, items_per_w, (bad.size, NO_MAX_ITEMS))
    q = rng.integers(1, 11, (no.size, NO_MAX_ITEMS))
    items = np.where(live, items, 0)
    q = np.where(live, q, 0)
    if rollback_frac > 0 and no.size:
        rb = np.nonzero(rng.random(no.size) < rollback_frac)[0]
        items[rb, k[rb] - 1] = items_per_w
    params[3, no] = k
    params[4:4 + NO_MAX_ITEMS, no] = items.T
    params[4 + NO_MAX_ITEMS:, no] = q.T
    pay = np.nonzero(kind == 1)[0]
    params[3, pay] = rng.integers(1, 5001, pay.size)
    return Bulk(types, params, np.arange(ts0, ts0 + n, dtype=np.int64))


def config3(n: int = 1 << 18, n_wh: int = 16, d_per_w: int = 10, c_per_d: int = 3000,
            items_per_w: int = 100_000, root_key: bool = False) -> Workload:
    rng_t = rng_for(3, 0)
    rng_b = rng_for(3, 1)
    bulk = order_bulk(rng_b, n, n_wh, d_per_w, c_per_d, items_per_w)
    n_no = int((bulk.type == 1).sum())
    n_lines = int(bulk.params[3][bulk.type == 1].sum())
    tabs = order_tables(rng_t, n_wh, d_per_w, c_per_d, items_per_w,
                        orders_capacity=max(n_no, 1), lines_capacity=max(n_lines, 1))
    return Workload(f"order-entry-{n_wh}w-n{n}", tabs, order_types(root_key), [bulk],
                    1 + NO_MAX_ITEMS,
                    meta=dict(n_wh=n_wh, d_per_w=d_per_w, c_per_d=c_per_d,
                              items_per_w=items_per_w))


# ---------------------------------------------------------------------------
# subscriber / call forwarding (TM-1 stand-in)

SUB_MIX = (0.60, 0.20, 0.08, 0.08, 0.02, 0.02)  # GET_SUB, GET_CF, UPD_SUB_FIELD, UPD_LOC, INS_CF, DEL_CF


def sub_tables(rng: np.random.Generator, n_sub: int, occupancy: float = 25 / 120) -> Dict[str, Table]:
    """Subscriber rows (int64 id, 4 int32 bit/byte fields, 10 int32 locations)
    and direct-addressed call-forwarding slots (occupied, end, number);
    slot = sid * 12 + cf_type * 3 + start_index."""
    cols = [np.arange(n_sub, dtype=np.int64)]
    cols += [rng.integers(0, 256, n_sub, dtype=np.int64).astype(np.int32) for _ in range(SUB_FIELDS)]
    cols += [rng.integers(-2**31, 2**31, n_sub, dtype=np.int64).astype(np.int32)
             for _ in range(SUB_LOCS)]
    sub = Table("subscriber", ["i64"] + ["i32"] * (SUB_FIELDS + SUB_LOCS), cols, n_sub, n_sub,
                root="subscriber", root_div=1)
    n_slot = n_sub * CF_SLOTS
    occ = (rng.random(n_slot) < occupancy).astype(np.int32)
    end = np.where(occ == 1, rng.integers(1, 25, n_slot), 0).astype(np.int32)
    num = np.where(occ == 1, rng.integers(0, 10**15, n_slot, dtype=np.int64), 0).astype(np.int64)
    cf = Table("call_fwd", ["i32", "i32", "i64"], [occ, end, num], n_slot, n_slot,
               root="subscriber", root_div=CF_SLOTS)
    return {"subscriber": sub, "call_fwd": cf}


def sub_types(root_key: bool = False) -> List[TypeDesc]:
    return [
        TypeDesc(4, "GET_SUB", 1, SUB_FIELDS + SUB_LOCS, SUB_ROLES, root_key=root_key),
        TypeDesc(5, "GET_CF", 2, 3, SUB_ROLES, root_key=root_key),
        TypeDesc(6, "UPD_SUB_FIELD", 3, 1, SUB_ROLES, root_key=root_key),
        TypeDesc(7, "UPD_LOC", 3, 1, SUB_ROLES, root_key=root_key),
        TypeDesc(8, "INS_CF", 4, 1, SUB_ROLES, root_key=root_key),
        TypeDesc(9, "DEL_CF", 2, 3, SUB_ROLES, root_key=root_key),
    ]


def sub_bulk(rng: np.random.Generator, n: int, n_sub: int, theta: float = 0.8,
             ts0: int = 0, mix=SUB_MIX) -> Bulk:
    """Subscriber mix; params: p0 = sid, p1 = field / location / slot index,
    p2 = new value or end time, p3 = forwarding number."""
    kind = rng.choice(len(mix), size=n, p=np.asarray(mix, dtype=np.float64))
    types = (kind + 4).astype(np.int32)
    params = np.zeros((4, n), dtype=np.int64)
    params[0] = zipf_ids(rng, n_sub, theta, n)
    sel = rng.integers(0, 1 << 30, n)
    params[1] = np.select([kind == 2, kind == 3], [sel % SUB_FIELDS, sel % SUB_LOCS], sel % CF_SLOTS)
    params[1][kind == 0] = 0
    params[2] = np.where(kind == 2, rng.integers(0, 256, n),
                         np.where(kind == 3, rng.integers(-2**31, 2**31, n),
                                  np.where(kind == 4, rng.integers(1, 25, n), 0)))
    params[3] = np.where(kind == 4, rng.integers(0, 10**15, n, dtype=np.int64), 0)
    return Bulk(types, params, np.arange(ts0, ts0 + n, dtype=np.int64))


def config5(n: int = 100_000, n_sub: int = 10_000_000, theta: float = 0.8) -> Workload:
    rng_t = rng_for(5, 0)
    rng_b = rng_for(5, 1)
    tabs = sub_tables(rng_t, n_sub)
    bulk = sub_bulk(rng_b, n, n_sub, theta)
    return Workload(f"subscriber-{n_sub}-n{n}", tabs, sub_types(), [bulk], SUB_FIELDS + SUB_LOCS,
                    meta=dict(n_sub=n_sub, theta=theta))


def poisson_arrivals(rng: np.random.Generator, rate_per_s: float, duration_s: float) -> np.ndarray:
    """Arrival times in nanoseconds of a Poisson process of the given rate."""
    n_est = int(rate_per_s * duration_s * 1.1) + 64
    gaps = rng.exponential(1e9 / rate_per_s, n_est)
    t = np.cumsum(gaps)
    return t[t < duration_s * 1e9].astype(np.int64)


# ---------------------------------------------------------------------------
# batching workload: many uneven bulks over two databases

def config4(n_bulks: int = 512, lo: int = 256, hi: int = 262_144, scale: float = 1.0,
            bank_branches: int = 64, accounts_per_branch: int = 100_000, n_wh: int = 16,
            items_per_w: int = 100_000, c_per_d: int = 3000):
    """512 bulks, sizes round(exp(U[ln lo, ln hi])) * scale; each bulk is a bank
    bulk (theta from {0, 0.8, 0.99}) or an order-entry bulk by coin flip.
    Timestamps increase globally across bulks.  Returns (bank Workload,
    order Workload, list of (db, bulk index)) in submission order."""
    rng = rng_for(4, 0)
    sizes = np.maximum(1, np.round(np.exp(rng.uniform(math.log(lo), math.log(hi), n_bulks))
                                   * scale)).astype(np.int64)
    which = rng.integers(0, 2, n_bulks)
    thetas = np.array([0.0, 0.8, 0.99])[rng.integers(0, 3, n_bulks)]
    rng_t = rng_for(4, 1)
    rng_b = rng_for(4, 2)
    n_bank_txn = int(sizes[which == 0].sum())
    bank_tabs = bank_tables(rng_t, bank_branches, bank_branches * 10,
                            bank_branches * accounts_per_branch, history_capacity=max(1, n_bank_txn))
    bank_bulks, order_bulks, order = [], [], []
    ts = 0
    for i in range(n_bulks):
        n = int(sizes[i])
        if which[i] == 0:
            b = bank_bulk(rng_b, n, bank_branches, bank_branches * 10,
                          bank_branches * accounts_per_branch, float(thetas[i]), ts0=ts)
            order.append(("bank", len(bank_bulks)))
            bank_bulks.append(b)
        else:
            b = order_bulk(rng_b, n, n_wh, 10, c_per_d, items_per_w, ts0=ts)
            order.append(("order", len(order_bulks)))
            order_bulks.append(b)
        ts += n
    n_no = sum(int((b.type == 1).sum()) for b in order_bulks)
    n_lines = sum(int(b.params[3][b.type == 1].sum()) for b in order_bulks)
    ord_tabs = order_tables(rng_t, n_wh, 10, c_per_d, items_per_w,
                            orders_capacity=max(1, n_no), lines_capacity=max(1, n_lines))
    bank = Workload("bank-batched", bank_tabs, bank_types(), bank_bulks, 3,
                    meta=dict(n_branch=bank_branches))
    orders = Workload("order-batched", ord_tabs, order_types(), order_bulks, 1 + NO_MAX_ITEMS,
                      meta=dict(n_wh=n_wh))
    return bank, orders, order


def shuffled(bulk: Bulk, rng: np.random.Generator, gapped: bool = False) -> Bulk:
    """The same transactions in a random input order; with ``gapped`` the
    timestamps are also spread over int64 with random gaps (order kept)."""
    perm = rng.permutation(bulk.n)
    ts = bulk.ts.copy()
    if gapped:
        gaps = rng.integers(1, 1 << 40, bulk.n, dtype=np.int64)
        ts = np.cumsum(gaps) - (1 << 62)
    return Bulk(bulk.type[perm].copy(), np.ascontiguousarray(bulk.params[:, perm]), ts[perm].copy())
