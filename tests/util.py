"""Shared test helpers (no method arithmetic beyond closed forms used as pins)."""
from __future__ import annotations

import numpy as np

from paper_1103_3105_amd import workloads as wl


def sizes_of(tables):
    return {k: v.n_rows for k, v in tables.items()}


def roots_of(tables):
    """table -> (root table, rows per root key) for tables that have a root."""
    return {k: (v.root, v.root_div) for k, v in tables.items() if v.root_div > 0}


def seg_inclusive_prefix(keys: np.ndarray, vals: np.ndarray) -> np.ndarray:
    """out[i] = sum of vals[j] over j <= i with keys[j] == keys[i] (arrays in
    timestamp order), computed with a stable sort and cumulative sums."""
    n = keys.shape[0]
    order = np.lexsort((np.arange(n), keys))
    ks, vs = keys[order], vals[order].astype(np.int64)
    cs = np.cumsum(vs)
    start = np.r_[True, ks[1:] != ks[:-1]] if n else np.zeros(0, bool)
    seg = np.cumsum(start) - 1
    base = (cs - vs)[np.flatnonzero(start)][seg]
    out = np.empty(n, dtype=np.int64)
    out[order] = cs - base
    return out


def small_bank(seed: int, n: int, n_branch=2, tpb=2, apt=3, theta=0.0):
    rng = np.random.default_rng(seed)
    tabs = wl.bank_tables(rng, n_branch, n_branch * tpb, n_branch * tpb * apt, history_capacity=n)
    bulk = wl.bank_bulk(rng, n, n_branch, n_branch * tpb, n_branch * tpb * apt, theta)
    return tabs, wl.bank_types(), bulk


def small_order(seed: int, n: int, n_wh=2, d_per_w=2, c_per_d=3, items_per_w=20, rollback_frac=0.0):
    """Order-entry bulk; rollback_frac > 0 registers new-order as the procedure
    that is not two-phase and makes that fraction of new-orders roll back."""
    rng = np.random.default_rng(seed)
    bulk = wl.order_bulk(rng, n, n_wh, d_per_w, c_per_d, items_per_w, rollback_frac=rollback_frac)
    n_no = int((bulk.type == 1).sum())
    n_l = int(bulk.params[3][bulk.type == 1].sum())
    tabs = wl.order_tables(rng, n_wh, d_per_w, c_per_d, items_per_w, max(n_no, 1), max(n_l, 1))
    return tabs, wl.order_types(rollback=rollback_frac > 0), bulk


def small_sub(seed: int, n: int, n_sub=5, theta=0.8):
    rng = np.random.default_rng(seed)
    tabs = wl.sub_tables(rng, n_sub, occupancy=0.5)
    bulk = wl.sub_bulk(rng, n, n_sub, theta)
    return tabs, wl.sub_types(), bulk


def copy_tables(tabs):
    return {k: v.copy() for k, v in tabs.items()}


def tables_equal(a, b, append_sort_col=None):
    """Compare two role->Table dicts column by column over the used rows."""
    for k in a:
        ta, tb = a[k], b[k]
        if ta.n_rows != tb.n_rows:
            return False, f"{k}: n_rows {ta.n_rows} != {tb.n_rows}"
        for c, (x, y) in enumerate(zip(ta.cols, tb.cols)):
            x, y = x[:ta.n_rows], y[:tb.n_rows]
            if ta.append and append_sort_col is not None:
                ox = np.lexsort(tuple(col[:ta.n_rows] for col in reversed(ta.cols)))
                oy = np.lexsort(tuple(col[:tb.n_rows] for col in reversed(tb.cols)))
                x, y = x[ox], y[oy]
            if not np.array_equal(x, y):
                bad = np.flatnonzero(x != y)[:5]
                return False, f"{k}.col{c} differs at rows {bad.tolist()}"
    return True, ""
