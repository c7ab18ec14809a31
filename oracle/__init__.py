"""Serial oracle for bulk transaction execution -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU engine never calls it and
shares no code with it.

* ``run_serial``  -- the C serial executor (``serial.c``): Definition 1
  (Section 3.1) written out, timed as the CPU baseline.
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
     "UPD_SUB_FIELD", "UPD_LOC", "INS_CF", "DEL_CF"))}
OK, E_ARG, E_DUP_TS, E_CAPACITY = 0, -1, -3, -4
COMMIT, ABORT, INVALID = 0, 1, 2


class _Table(ctypes.Structure):
    _fields_ = [("col", ctypes.c_void_p * 16), ("n_rows", ctypes.c_int64),
                ("capacity", ctypes.c_int64)]


def build(force: bool = False) -> str:
    """Compile serial.c into liboracle.so (plain gcc, host only)."""
    src = os.path.join(_HERE, "serial.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < max(
            os.path.getmtime(src), os.path.getmtime(os.path.join(_HERE, "oracle.h"))):
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
                               "-o", _LIB_PATH, src])
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
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def run_serial(tables: Dict[str, object], types: Sequence[object], type_arr: np.ndarray,
               params: np.ndarray, ts: np.ndarray, width: int):
    """Execute one bulk serially in timestamp order, mutating ``tables``.

    ``types``: objects with ``type_id`` and ``proc`` (procedure name).
    Returns (rc, status[n] int32, results[n, width] int64).  On rc != 0 no
    table was touched.
    """
    lib = _load()
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
    status = np.zeros(n, dtype=np.int32)
    results = np.zeros((n, width), dtype=np.int64)
    rc = lib.orc_execute(n, _ptr(type_arr), _ptr(params), int(params.shape[0]), _ptr(ts),
                         _ptr(pot), int(n_types), arr, _ptr(status), _ptr(results), int(width))
    if rc == OK:
        for i, role in enumerate(ROLES):
            t = tables.get(role)
            if t is not None:
                t.n_rows = int(arr[i].n_rows)
    return rc, status, results
