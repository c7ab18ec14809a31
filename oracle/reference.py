"""Pure-Python references for the dependency analysis -- TEST INFRASTRUCTURE.

Everything here is plain and slow; it is meant for bulks of up to a few
thousand transactions (the rank and depth helpers use numpy and scale to a
few million operations).

Contents
--------
* ``basic_ops``       -- the basic operations of one transaction: reads and
  writes on data items (Section 4.1).  A read-modify-write is one write; an
  item accessed twice by one transaction is one operation, a write if any
  access writes.  Items are (table, row); in root-key mode every item is
  replaced by its partition root (Section 5.1, lock on the primary key of the
  root relation) -- a coarsening, which keeps every conflict (Appendix B).
* ``paper_ranks``     -- the rank rule of Section 4.2 on (item, id)-sorted ops.
* ``depth_*``         -- transaction depth in the T-dependency graph
  (Section 4.1) four ways: pairwise definition with conditions (a)-(c) plus
  longest path, Appendix B construction plus topological sort (Section 4.2),
  an O(ops) per-item scan, and Kahn levels.
* ``features`` / ``choose_strategy`` -- w0, d and c of Appendix D, and
  Algorithm 1.
* ``py_execute``      -- serial twin of the C oracle that runs the
  transactions in any given order (for brute force over linear extensions).
"""
from __future__ import annotations

import itertools
from typing import Dict, List, Sequence, Tuple

import numpy as np

NO_MAX_ITEMS = 15
CF_SLOTS = 12
SUB_FIELDS = 4
SUB_LOCS = 10
COMMIT, ABORT, INVALID = 0, 1, 2


# ---------------------------------------------------------------------------
# schema helpers

def _dims(sizes: Dict[str, int]):
    nw = sizes.get("warehouse", 0)
    nd = sizes.get("district", 0)
    if nw <= 0 or nd <= 0:
        return None
    return dict(nw=nw, dpw=nd // nw, cpd=sizes.get("customer", 0) // nd,
                ipw=sizes.get("stock", 0) // nw)


def _in(v, n):
    return 0 <= v < n


def valid(proc: str, p: Sequence[int], sizes: Dict[str, int]) -> bool:
    """Parameter validity; an invalid transaction has no effect."""
    i32 = lambda v: -2**31 <= v < 2**31
    if proc == "DEBIT_CREDIT":
        return (_in(p[0], sizes.get("account", 0)) and _in(p[1], sizes.get("teller", 0))
                and _in(p[2], sizes.get("branch", 0)))
    if proc in ("NEW_ORDER", "NEW_ORDER_RB", "PAYMENT", "ORDER_STATUS"):
        d = _dims(sizes)
        if d is None or not (_in(p[0], d["nw"]) and _in(p[1], d["dpw"]) and _in(p[2], d["cpd"])):
            return False
        if proc not in ("NEW_ORDER", "NEW_ORDER_RB"):
            return True
        k = p[3]
        if not 1 <= k <= NO_MAX_ITEMS:
            return False
        # the variant that is not two-phase also names the unused item id ipw
        items = d["ipw"] + (1 if proc == "NEW_ORDER_RB" else 0)
        return all(_in(p[4 + j], items) and 1 <= p[4 + NO_MAX_ITEMS + j] <= 1000
                   for j in range(k))
    ns = sizes.get("subscriber", 0)
    if proc == "GET_SUB":
        return _in(p[0], ns)
    if proc in ("GET_CF", "DEL_CF"):
        return _in(p[0], ns) and _in(p[1], CF_SLOTS)
    if proc == "UPD_SUB_FIELD":
        return _in(p[0], ns) and _in(p[1], SUB_FIELDS) and i32(p[2])
    if proc == "UPD_LOC":
        return _in(p[0], ns) and _in(p[1], SUB_LOCS) and i32(p[2])
    if proc == "INS_CF":
        return _in(p[0], ns) and _in(p[1], CF_SLOTS) and i32(p[2])
    return False


def raw_accesses(proc: str, p: Sequence[int], sizes: Dict[str, int]) -> List[Tuple[str, int, bool]]:
    """(table, row, is_write) for every access of a valid transaction, in
    procedure order; appends to append-only tables are not data items that
    any transaction reads, so they are not listed."""
    if proc == "DEBIT_CREDIT":
        return [("account", p[0], True), ("teller", p[1], True), ("branch", p[2], True)]
    if proc in ("NEW_ORDER", "NEW_ORDER_RB", "PAYMENT", "ORDER_STATUS"):
        d = _dims(sizes)
        drow = p[0] * d["dpw"] + p[1]
        crow = drow * d["cpd"] + p[2]
        if proc in ("NEW_ORDER", "NEW_ORDER_RB"):   # the unused item has no row
            return [("stock", p[0] * d["ipw"] + p[4 + j], True) for j in range(p[3])
                    if p[4 + j] < d["ipw"]]
        if proc == "PAYMENT":
            return [("warehouse", p[0], True), ("district", drow, True), ("customer", crow, True)]
        return [("customer", crow, False)]
    if proc == "GET_SUB":
        return [("subscriber", p[0], False)]
    if proc == "GET_CF":
        return [("call_fwd", p[0] * CF_SLOTS + p[1], False)]
    if proc in ("UPD_SUB_FIELD", "UPD_LOC"):
        return [("subscriber", p[0], True)]
    if proc in ("INS_CF", "DEL_CF"):
        return [("call_fwd", p[0] * CF_SLOTS + p[1], True)]
    raise ValueError(proc)


def basic_ops(proc: str, p: Sequence[int], sizes: Dict[str, int], root_key: bool = False,
              roots: Dict[str, Tuple[str, int]] = None) -> Dict[Tuple[str, int], bool]:
    """item -> is_write, deduplicated (write wins).  ``roots``: table ->
    (root table, rows per root key), used in root-key mode."""
    ops: Dict[Tuple[str, int], bool] = {}
    for tab, row, w in raw_accesses(proc, p, sizes):
        item = (tab, int(row))
        if root_key:
            rt, div = roots[tab]
            item = (rt, int(row) // div)
        ops[item] = ops.get(item, False) or w
    return ops


def bulk_ops(types, type_arr, params, ts, sizes, roots=None):
    """Per transaction in timestamp order: (input index, proc, ops dict).
    Invalid or unregistered transactions get no ops."""
    by_id = {t.type_id: t for t in types}
    order = np.argsort(ts, kind="stable")
    out = []
    for i in order:
        i = int(i)
        t = by_id.get(int(type_arr[i]))
        p = [int(x) for x in params[:, i]]
        p += [0] * max(0, 4 + 2 * NO_MAX_ITEMS - len(p))
        if t is None or not valid(t.proc, p, sizes):
            out.append((i, None, {}))
            continue
        out.append((i, t.proc, basic_ops(t.proc, p, sizes, t.root_key, roots)))
    return out


# ---------------------------------------------------------------------------
# rank rule and depth

def paper_ranks(txn_ops: List[Dict]) -> Tuple[List[Tuple], np.ndarray, np.ndarray]:
    """Section 4.2: group the basic operations by item, order each group by
    timestamp (here: position in ``txn_ops``); the first op of a group has
    rank 0; op i has rank r(i-1) + 1 if it or op i-1 writes, else r(i-1).
    Returns (sorted ops [(item, pos, w)], rank per sorted op, per-transaction
    maximum rank)."""
    flat = [(item, pos, w) for pos, ops in enumerate(txn_ops) for item, w in ops.items()]
    flat.sort(key=lambda x: (x[0], x[1]))
    ranks = np.zeros(len(flat), dtype=np.int64)
    maxrank = np.zeros(len(txn_ops), dtype=np.int64)
    for i, (item, pos, w) in enumerate(flat):
        if i == 0 or flat[i - 1][0] != item:
            ranks[i] = 0
        else:
            ranks[i] = ranks[i - 1] + (1 if (w or flat[i - 1][2]) else 0)
        maxrank[pos] = max(maxrank[pos], ranks[i])
    return flat, ranks, maxrank


def conflict(a: Dict, b: Dict) -> bool:
    """Two transactions conflict iff they touch a common item and at least
    one of the two accesses writes (Section 4.1)."""
    return any(it in b and (w or b[it]) for it, w in a.items())


def tdg_edges_pairwise(txn_ops: List[Dict]) -> List[Tuple[int, int]]:
    """Edges t1 -> t2 by conditions (a) conflict, (b) ts1 < ts2, (c) no t
    between them conflicting with both (Section 4.1).  O(n^3)."""
    n = len(txn_ops)
    C = [[conflict(txn_ops[i], txn_ops[j]) for j in range(n)] for i in range(n)]
    edges = []
    for i in range(n):
        for j in range(i + 1, n):
            if C[i][j] and not any(C[i][k] and C[k][j] for k in range(i + 1, j)):
                edges.append((i, j))
    return edges


def longest_path_depth(n: int, edges: Sequence[Tuple[int, int]]) -> np.ndarray:
    """Depth of every vertex: longest path from a source (sources: 0).
    Vertices are numbered in timestamp order, so every edge goes forward and
    increasing index is a topological order (Section 4.2)."""
    preds: List[List[int]] = [[] for _ in range(n)]
    for a, b in edges:
        preds[b].append(a)
    depth = np.zeros(n, dtype=np.int64)
    for v in range(n):
        if preds[v]:
            depth[v] = 1 + max(depth[u] for u in preds[v])
    return depth


def depth_pairwise(txn_ops: List[Dict]) -> np.ndarray:
    return longest_path_depth(len(txn_ops), tdg_edges_pairwise(txn_ops))


def tdg_edges_appendix_b(txn_ops: List[Dict]) -> List[Tuple[int, int]]:
    """Appendix B: add transactions in timestamp order; per item keep the list
    of transactions that accessed it.  A write scans back from the tail to the
    last writer t_w: if t_w is the tail the edge is t_w -> t, otherwise edges
    from every reader between t_w and the tail.  A read adds t_w -> t.  (With
    no writer in the list, a write takes edges from every reader in it.)"""
    lists: Dict = {}
    edges = set()
    for t, ops in enumerate(txn_ops):
        for item, w in ops.items():
            lst = lists.setdefault(item, [])
            if lst:
                k = len(lst) - 1
                while k >= 0 and not lst[k][1]:
                    k -= 1
                if w:
                    if k == len(lst) - 1:
                        edges.add((lst[k][0], t))
                    else:
                        for u, _ in lst[k + 1:]:
                            edges.add((u, t))
                elif k >= 0:
                    edges.add((lst[k][0], t))
            lst.append((t, w))
    return sorted(edges)


def depth_appendix_b(txn_ops: List[Dict]) -> np.ndarray:
    return longest_path_depth(len(txn_ops), tdg_edges_appendix_b(txn_ops))


def depth_scan(txn_ops: List[Dict]) -> np.ndarray:
    """O(ops) scan in timestamp order: a read depends on the last write of its
    item; a write depends on the last write and on every read since it."""
    last_w: Dict = {}      # item -> depth of last writer
    reads_since: Dict = {}  # item -> max depth of readers since last write
    depth = np.zeros(len(txn_ops), dtype=np.int64)
    for t, ops in enumerate(txn_ops):
        d = -1
        for item, w in ops.items():
            if item in last_w:
                d = max(d, last_w[item])
            if w and item in reads_since:
                d = max(d, reads_since[item])
        depth[t] = d + 1
        for item, w in ops.items():
            if w:
                last_w[item] = depth[t]
                reads_since.pop(item, None)
            else:
                reads_since[item] = max(reads_since.get(item, -1), depth[t])
    return depth


def kahn_levels(txn_ops: List[Dict]) -> List[List[int]]:
    """Repeatedly take every transaction with no undone conflicting
    predecessor (the 0-set), remove it, and continue (Section 5.3)."""
    edges = tdg_edges_appendix_b(txn_ops)
    n = len(txn_ops)
    indeg = np.zeros(n, dtype=np.int64)
    succ: List[List[int]] = [[] for _ in range(n)]
    for a, b in edges:
        indeg[b] += 1
        succ[a].append(b)
    frontier = [v for v in range(n) if indeg[v] == 0]
    levels = []
    while frontier:
        levels.append(sorted(frontier))
        nxt = []
        for v in frontier:
            for s in succ[v]:
                indeg[s] -= 1
                if indeg[s] == 0:
                    nxt.append(s)
        frontier = nxt
    return levels


# ---------------------------------------------------------------------------
# features and Algorithm 1

def partitions_of(ops: Dict, roots: Dict[str, Tuple[str, int]], part_size: int) -> set:
    """Partition ids of a transaction's items: root key // partition size.
    Items already replaced by their root (root-key mode) map directly."""
    out = set()
    for (tab, row) in ops:
        rt, div = roots[tab]
        out.add((row // div) // part_size)
    return out


def features(txn_ops: List[Dict], roots, part_size: int = 1):
    """(w0, d, c): size of the 0-set (transactions with operations and no
    conflicting predecessor), depth computed as the maximum paper rank
    (Section 4.2 step 5), and the number of transactions whose items span more
    than one partition (Appendix D)."""
    _, _, maxrank = paper_ranks(txn_ops)
    live = np.array([len(o) > 0 for o in txn_ops], dtype=bool)   # invalid txns have no ops
    w0 = int(((maxrank == 0) & live).sum())
    d = int(maxrank.max()) if len(maxrank) else 0
    c = sum(1 for ops in txn_ops if len(partitions_of(ops, roots, part_size)) > 1)
    return w0, d, c


def choose_strategy(w0: int, d: int, c: int, w0_bar: int, c_bar: int, d_bar: int) -> str:
    """Algorithm 1 (Appendix D)."""
    if w0 >= w0_bar:
        return "KSET"
    if c <= c_bar or d >= d_bar:
        return "PART"
    return "TPL"


def strategy_run(chosen: str, c: int) -> str:
    """The executor that runs once a strategy is chosen or requested: PART
    needs every transaction inside one partition, and Section 5.2 hands
    bulks with cross-partition transactions to TPL."""
    return "TPL" if chosen == "PART" and c > 0 else chosen


# ---------------------------------------------------------------------------
# serial twin (any order)

def _i32(v: int) -> int:
    v &= 0xFFFFFFFF
    return v - (1 << 32) if v >= 1 << 31 else v


def _i64(v: int) -> int:
    v &= 0xFFFFFFFFFFFFFFFF
    return v - (1 << 64) if v >= 1 << 63 else v


def py_execute(tables: Dict[str, object], types, type_arr, params, ts, width: int, order=None):
    """Run the transactions one by one in ``order`` (input indices; default:
    increasing timestamp), mutating ``tables``.  Returns (status, results)."""
    by_id = {t.type_id: t for t in types}
    n = len(type_arr)
    if order is None:
        order = [int(i) for i in np.argsort(ts, kind="stable")]
    sizes = {k: v.n_rows for k, v in tables.items()}
    status = np.zeros(n, dtype=np.int32)
    results = np.zeros((n, width), dtype=np.int64)
    for i in order:
        t = by_id.get(int(type_arr[i]))
        p = [int(x) for x in params[:, i]] + [0] * 40
        if t is None or not valid(t.proc, p, sizes):
            status[i] = INVALID
            continue
        res = [0] * 64
        st = COMMIT
        proc = t.proc
        if proc == "DEBIT_CREDIT":
            A, T, B = tables["account"].cols[0], tables["teller"].cols[0], tables["branch"].cols[0]
            A[p[0]] = _i64(int(A[p[0]]) + p[3])
            T[p[1]] = _i64(int(T[p[1]]) + p[3])
            B[p[2]] = _i64(int(B[p[2]]) + p[3])
            H = tables["history"]
            for c, v in enumerate((p[0], p[1], p[2], p[3], int(ts[i]))):
                H.cols[c][H.n_rows] = v
            H.n_rows += 1
            res[:3] = [int(A[p[0]]), int(T[p[1]]), int(B[p[2]])]
        elif proc == "NEW_ORDER_RB" and any(p[4 + j] == _dims(sizes)["ipw"] for j in range(p[3])):
            st = ABORT   # rolled back: no effect, results 0 (Appendix D)
        elif proc in ("NEW_ORDER", "NEW_ORDER_RB", "PAYMENT", "ORDER_STATUS"):
            d = _dims(sizes)
            drow = p[0] * d["dpw"] + p[1]
            crow = drow * d["cpd"] + p[2]
            if proc in ("NEW_ORDER", "NEW_ORDER_RB"):
                S = tables["stock"].cols[0]
                L, O = tables["order_line"], tables["orders"]
                res[0] = p[3]
                for j in range(p[3]):
                    item, q = p[4 + j], p[4 + NO_MAX_ITEMS + j]
                    row = p[0] * d["ipw"] + item
                    s = int(S[row]) - q
                    if s < 10:
                        s += 91
                    S[row] = _i32(s)
                    res[1 + j] = int(S[row])
                    for c, v in enumerate((int(ts[i]), j, item, q, p[0])):
                        L.cols[c][L.n_rows] = v
                    L.n_rows += 1
                for c, v in enumerate((int(ts[i]), p[0], p[1], p[2], p[3])):
                    O.cols[c][O.n_rows] = v
                O.n_rows += 1
            elif proc == "PAYMENT":
                Wb, Db, Cb = (tables[x].cols[0] for x in ("warehouse", "district", "customer"))
                Wb[p[0]] = _i64(int(Wb[p[0]]) + p[3])
                Db[drow] = _i64(int(Db[drow]) + p[3])
                Cb[crow] = _i64(int(Cb[crow]) + p[3])
                res[:3] = [int(Wb[p[0]]), int(Db[drow]), int(Cb[crow])]
            else:
                res[0] = int(tables["customer"].cols[0][crow])
        else:
            S = tables["subscriber"].cols
            C = tables["call_fwd"].cols
            slot = p[0] * CF_SLOTS + p[1]
            if proc == "GET_SUB":
                res[:SUB_FIELDS + SUB_LOCS] = [int(S[1 + f][p[0]]) for f in range(SUB_FIELDS + SUB_LOCS)]
            elif proc == "GET_CF":
                res[:3] = [int(C[0][slot]), int(C[1][slot]), int(C[2][slot])]
            elif proc in ("UPD_SUB_FIELD", "UPD_LOC"):
                col = S[1 + p[1] + (SUB_FIELDS if proc == "UPD_LOC" else 0)]
                res[0] = int(col[p[0]])
                col[p[0]] = _i32(p[2])
            elif proc == "INS_CF":
                res[0] = int(C[0][slot])
                if C[0][slot]:
                    st = ABORT
                else:
                    C[0][slot], C[1][slot], C[2][slot] = 1, _i32(p[2]), p[3]
            elif proc == "DEL_CF":
                if not C[0][slot]:
                    st = ABORT
                else:
                    res[:3] = [1, int(C[1][slot]), int(C[2][slot])]
                    C[0][slot], C[1][slot], C[2][slot] = 0, 0, 0
        status[i] = st
        results[i] = res[:width]
    return status, results


def linear_extensions(txn_ops: List[Dict], limit: int = 100000):
    """Every order of the transactions (by timestamp position) that keeps each
    conflicting pair in timestamp order; n <= 7."""
    n = len(txn_ops)
    C = [[conflict(txn_ops[i], txn_ops[j]) for j in range(n)] for i in range(n)]
    count = 0
    for perm in itertools.permutations(range(n)):
        where = {v: k for k, v in enumerate(perm)}
        if all(where[i] < where[j] for i in range(n) for j in range(i + 1, n) if C[i][j]):
            yield list(perm)
            count += 1
            if count >= limit:
                return
