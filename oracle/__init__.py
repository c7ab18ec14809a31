"""Serial oracle for bulk transaction execution -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU engine never calls it and
shares no code with it.

* ``run_serial``  -- the C serial executor (``serial.c``): Definition 1
  (Section 3.1) written out, timed as the CPU baseline.
* ``run_partitioned`` / ``partition_ids`` -- the paper's CPU counterpart
  (``partitioned.c``, Section 6.3): H-Store-style workers, one per group of
  partitions, on all host cores; bit-exact with ``run_serial``.
* ``reference``   -- pure-Python pieces: a serial twin that can run any order
  (for brute force over linear extensions), the per-procedure basic
  operations (Section 4.1), the paper's rank rule (Section 4.2), depth by four
  independent methods (Sections 4.1-4.2, Appendix B), the structural features
  of Appendix D and Algorithm 1.

Tables are passed duck-typed: anything with ``cols`` (list of numpy arrays),
``n_rows`` and ``capacity``, keyed by role name.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

ROLES = ("account", "teller", "branch", "history", "warehouse", "district", "customer",
         "stock", "orders", "order_line", "subscriber", "call_fwd")
PROC_ID = {name: i + 1 for i, name in enumerate(
    ("DEBIT_CREDIT", "NEW_ORDER", "PAYMENT", "ORDER_STATUS", "GET_SUB", "GET_CF",
     "UPD_SUB_FIELD", "UPD_LOC", "INS_CF", "DEL_CF", "NEW_ORDER_RB"))}
OK, E_ARG, E_DUP_TS, E_CAPACITY = 0, -1, -3, -4
COMMIT, ABORT, INVALID = 0, 1, 2


class _Table(ctypes.Structure):
    _fields_ = [("col", ctypes.c_void_p * 16), ("n_rows", ctypes.c_int64),
                ("capacity", ctypes.c_int64)]


def build(force: bool = False) -> str:
    """Compile serial.c and partitioned.c into liboracle.so (plain gcc, host only)."""
    srcs = [os.path.join(_HERE, f) for f in ("serial.c", "partitioned.c")]
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < max(
            [os.path.getmtime(s) for s in srcs] + [os.path.getmtime(os.path.join(_HERE, "oracle.h"))]):
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
                               "-o", _LIB_PATH + ".tmp", *srcs, "-lpthread"])
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.orc_execute.restype = ctypes.c_int
        lib.orc_execute.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                    ctypes.POINTER(_Table), ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_int32]
        lib.orc_execute_partitioned.restype = ctypes.c_int
        lib.orc_execute_partitioned.argtypes = [
            ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(_Table), ctypes.c_void_p, ctypes.c_int32,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _marshal(tables, types, type_arr, params, ts):
    n = int(type_arr.shape[0])
    type_arr = np.ascontiguousarray(type_arr, dtype=np.int32)
    params = np.ascontiguousarray(params, dtype=np.int64)
    ts = np.ascontiguousarray(ts, dtype=np.int64)
    n_types = max([t.type_id for t in types] + [-1]) + 1
    pot = np.zeros(max(n_types, 1), dtype=np.int32)
    for t in types:
        pot[t.type_id] = PROC_ID[t.proc]
    arr = (_Table * len(ROLES))()
    for i, role in enumerate(ROLES):
        t = tables.get(role)
        if t is None:
            continue
        for c, col in enumerate(t.cols):
            assert col.flags.c_contiguous
            arr[i].col[c] = _ptr(col)
        arr[i].n_rows = t.n_rows
        arr[i].capacity = t.capacity
    return n, type_arr, params, ts, n_types, pot, arr


def _unmarshal(tables, arr):
    for i, role in enumerate(ROLES):
        t = tables.get(role)
        if t is not None:
            t.n_rows = int(arr[i].n_rows)


def run_serial(tables: Dict[str, object], types: Sequence[object], type_arr: np.ndarray,
               params: np.ndarray, ts: np.ndarray, width: int):
    """Execute one bulk serially in timestamp order, mutating ``tables``.

    ``types``: objects with ``type_id`` and ``proc`` (procedure name).
    Returns (rc, status[n] int32, results[n, width] int64).  On rc != 0 no
    table was touched.
    """
    lib = _load()
    n, type_arr, params, ts, n_types, pot, arr = _marshal(tables, types, type_arr, params, ts)
    status = np.zeros(n, dtype=np.int32)
    results = np.zeros((n, width), dtype=np.int64)
    rc = lib.orc_execute(n, _ptr(type_arr), _ptr(params), int(params.shape[0]), _ptr(ts),
                         _ptr(pot), int(n_types), arr, _ptr(status), _ptr(results), int(width))
    if rc == OK:
        _unmarshal(tables, arr)
    return rc, status, results


def partition_ids(tables: Dict[str, object], types: Sequence[object], type_arr: np.ndarray,
                  params: np.ndarray, part_size: int = 1) -> np.ndarray:
    """Partition of every transaction for the partitioned executor: the
    partition (root key // part_size, Section 5.2) that holds all of its rows,
    or -1 when its rows lie in several.  Tables name their root table and
    rows per root key (``root_div``); values for invalid transactions are
    arbitrary (they are never run)."""
    n = int(type_arr.shape[0])
    out = np.full(n, -1, dtype=np.int64)
    proc_of = {t.type_id: t.proc for t in types}
    for tid, proc in proc_of.items():
        if len(proc_of) == 1 and bool((type_arr == tid).all()):
            sel = slice(None)           # one type throughout: no gather
            p = [params[k] for k in range(min(params.shape[0], 3))]
        else:
            sel = np.flatnonzero(type_arr == tid)
            if sel.size == 0:
                continue
            p = [params[k][sel] for k in range(min(params.shape[0], 3))]

        def root(role, row):
            return row // max(tables[role].root_div, 1)
        if proc == "DEBIT_CREDIT":
            keys = [root("account", p[0]), root("teller", p[1]), root("branch", p[2])]
        elif proc in ("NEW_ORDER", "PAYMENT", "ORDER_STATUS"):
            # every row these touch sits under warehouse w (district, customer
            # and stock rows are numbered warehouse-major)
            keys = [root("warehouse", p[0])]
        else:   # subscriber procedures: the subscriber row and its call-forwarding slots
            keys = [root("subscriber", p[0])]
        pid = keys[0] // part_size
        for k in keys[1:]:
            pid = np.where((k // part_size) == pid, pid, -1)
        out[sel] = pid
    return out


def run_partitioned(tables: Dict[str, object], types: Sequence[object], type_arr: np.ndarray,
                    params: np.ndarray, ts: np.ndarray, width: int, part: np.ndarray,
                    n_threads: int):
    """The partitioned CPU counterpart on ``n_threads`` workers; same
    contract as ``run_serial`` (``part`` from ``partition_ids``)."""
    lib = _load()
    n, type_arr, params, ts, n_types, pot, arr = _marshal(tables, types, type_arr, params, ts)
    part = np.ascontiguousarray(part, dtype=np.int64)
    assert part.shape[0] == n
    status = np.zeros(n, dtype=np.int32)
    results = np.zeros((n, width), dtype=np.int64)
    rc = lib.orc_execute_partitioned(n, _ptr(type_arr), _ptr(params), int(params.shape[0]), _ptr(ts),
                                     _ptr(pot), int(n_types), arr, _ptr(part), int(n_threads),
                                     _ptr(status), _ptr(results), int(width))
    if rc == OK:
        _unmarshal(tables, arr)
    return rc, status, results


def run_sequence(tables: Dict[str, object], types: Sequence[object], bulks, times: int = 1):
    """Several bulks one after another, each serially in timestamp order
    (Definition 1 per bulk, bulks in the given order), mutating ``tables``.

    ``bulks``: (bulk, width) pairs, a bulk having ``type``, ``params`` and
    ``ts``.  ``times`` > 1 replays the whole sequence again on the resulting
    tables.  Returns the (status, results) of every bulk of the last pass."""
    out = []
    for _ in range(times):
        out = []
        for b, width in bulks:
            rc, st, res = run_serial(tables, types, b.type, b.params, b.ts, width)
            if rc != OK:
                raise RuntimeError(f"oracle rejected a bulk of the sequence: rc={rc}")
            out.append((st, res))
    return out
