"""Thin Python binding of the C ABI in include/gputx.h.

Only argument marshalling lives here: every step of a bulk runs in the HIP
kernels of libgputx.so.  torch provides device memory and streams.  There is
no fallback: if the library is missing, importing this module raises.

The functions keep the ABI's names (``gputx_create``, ``gputx_load_tables``,
``gputx_register_types``, ``gputx_workspace_size``, ``gputx_execute_bulk``,
``gputx_row_count`` ...).  ``Engine`` bundles them for one device database.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import c_int32, c_int64, c_void_p, c_size_t, POINTER
from typing import Dict, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgputx.so")

OK, E_ARG, E_TYPE, E_DUP_TS, E_CAPACITY, E_HIP, E_STATE, E_DEADLOCK, E_UNSORTED, E_INTERNAL = (
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9)
AUTO, TPL, PART, KSET = 0, 1, 2, 3
STRATEGY = {"AUTO": AUTO, "TPL": TPL, "PART": PART, "KSET": KSET}
STRATEGY_NAME = {v: k for k, v in STRATEGY.items()}
COMMIT, ABORT, INVALID = 0, 1, 2
I32, I64 = 1, 2
PROC = {"DEBIT_CREDIT": 1, "NEW_ORDER": 2, "PAYMENT": 3, "ORDER_STATUS": 4, "GET_SUB": 5,
        "GET_CF": 6, "UPD_SUB_FIELD": 7, "UPD_LOC": 8, "INS_CF": 9, "DEL_CF": 10, "NEW_ORDER_RB": 11}
MAX_TYPES, MAX_TABLES, MAX_COLS, MAX_ROLES = 16, 32, 16, 8


class Options(ctypes.Structure):
    _fields_ = [("w0_bar", c_int64), ("c_bar", c_int64), ("d_bar", c_int64),
                ("part_size", c_int64), ("group_by_type", c_int32), ("kset_narrow", c_int32),
                ("spin_limit_ms", c_int32), ("grid_blocks", c_int32), ("part_pipeline", c_int32),
                ("part_scan", c_int32), ("tpl_lanes", c_int32)]


class TableDesc(ctypes.Structure):
    _fields_ = [("table_id", c_int32), ("n_cols", c_int32), ("n_rows", c_int64),
                ("capacity", c_int64), ("append_only", c_int32), ("root_table_id", c_int32),
                ("root_div", c_int64), ("col_dtype", c_int32 * MAX_COLS),
                ("col_ptr", c_void_p * MAX_COLS)]


class TypeDesc(ctypes.Structure):
    _fields_ = [("type_id", c_int32), ("proc", c_int32), ("n_params", c_int32),
                ("n_results", c_int32), ("table_ids", c_int32 * MAX_ROLES),
                ("root_key", c_int32), ("single_partition", c_int32)]


class BulkDesc(ctypes.Structure):
    _fields_ = [("n", c_int64), ("type", c_void_p), ("params", c_void_p), ("n_params", c_int32),
                ("ts", c_void_p), ("ts_sorted", c_int32), ("max_ops", c_int32),
                ("type_mask", ctypes.c_uint32), ("reserved", c_int32)]


class BulkStats(ctypes.Structure):
    _fields_ = [("error", c_int32), ("chosen", c_int32), ("n_ops", c_int64), ("w0", c_int64),
                ("depth", c_int64), ("cross", c_int64), ("waves", c_int64),
                ("committed", c_int64), ("aborted", c_int64), ("invalid", c_int64),
                ("appended", c_int64), ("part_scan", c_int64),
                ("reserved", c_int64 * 6)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k in ("error", "chosen", "n_ops", "w0", "depth", "cross",
                                              "waves", "committed", "aborted", "invalid",
                                              "appended", "part_scan")}

    @property
    def label(self) -> str:
        """Name of the executor that ran: PART's per-cell map scan form is
        reported as PART-scan, apart from Section 5.2's sequential form."""
        name = STRATEGY_NAME.get(self.chosen, str(self.chosen))
        return "PART-scan" if name == "PART" and self.part_scan > 0 else name


STATS_BYTES = ctypes.sizeof(BulkStats)


class Trace(ctypes.Structure):
    _fields_ = [("n", c_int64), ("arrival_ns", c_void_p), ("type", c_void_p), ("params", c_void_p),
                ("n_params", c_int32), ("ts", c_void_p)]


class ServeOpts(ctypes.Structure):
    _fields_ = [("deadline_ns", c_int64), ("slots", c_int32), ("strategy", c_int32),
                ("max_bulk", c_int64), ("hbm_budget", c_int64), ("width", c_int32),
                ("max_ops", c_int32)]


class ServeBulk(ctypes.Structure):
    _fields_ = [("first", c_int64), ("count", c_int64), ("cut_ns", c_int64), ("issued_ns", c_int64),
                ("done_ns", c_int64), ("error", c_int32), ("slot", c_int32), ("front_us", c_int32),
                ("exec_us", c_int32)]


class ServeReport(ctypes.Structure):
    _fields_ = [("n_bulks", c_int64), ("committed", c_int64), ("aborted", c_int64),
                ("invalid", c_int64), ("elapsed_ns", c_int64), ("slots_used", c_int32),
                ("reserved", c_int32), ("slot_bytes", c_int64)]


class BatchItem(ctypes.Structure):
    _fields_ = [("bulk", BulkDesc), ("strategy", c_int32), ("lane", c_int32),
                ("workspace", c_void_p), ("ws_bytes", c_size_t), ("status_out", c_void_p),
                ("results_out", c_void_p), ("width", c_int32), ("stats", c_void_p),
                ("grid_blocks", c_int32), ("kset_narrow", c_int32)]


class PoolStats(ctypes.Structure):
    _fields_ = [("error", c_int32), ("reserved", c_int32), ("added", c_int64), ("done_prefix", c_int64),
                ("pending_ops", c_int64), ("waves", c_int64), ("executed", c_int64),
                ("committed", c_int64), ("aborted", c_int64), ("invalid", c_int64),
                ("last_width", c_int64), ("fetched", c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(the engine has no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    H = c_void_p
    sig = {
        "gputx_default_options": (c_int32, [POINTER(Options)]),
        "gputx_create": (c_int32, [c_int32, POINTER(Options), POINTER(H)]),
        "gputx_destroy": (c_int32, [H]),
        "gputx_set_options": (c_int32, [H, POINTER(Options)]),
        "gputx_load_tables": (c_int32, [H, POINTER(TableDesc), c_int32]),
        "gputx_register_types": (c_int32, [H, POINTER(TypeDesc), c_int32]),
        "gputx_workspace_size": (c_size_t, [H, c_int64]),
        "gputx_workspace_size_ops": (c_size_t, [H, c_int64, c_int32]),
        "gputx_execute_bulk": (c_int32, [H, POINTER(BulkDesc), c_int32, c_void_p, c_size_t,
                                         c_void_p, c_void_p, c_int32, c_void_p, c_void_p]),
        "gputx_execute_bulk_relaxed": (c_int32, [H, POINTER(BulkDesc), c_int32, c_void_p, c_size_t,
                                                 c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
        "gputx_execute_bulk_noalloc": (c_int32, [H, POINTER(BulkDesc), c_int32, c_void_p, c_void_p,
                                                 c_int32, c_void_p, c_void_p]),
        "gputx_row_count": (c_int32, [H, c_int32, POINTER(c_int64), c_void_p]),
        "gputx_set_row_count": (c_int32, [H, c_int32, c_int64, c_void_p]),
        "gputx_last_error": (ctypes.c_char_p, [H]),
        "gputx_phase_timing": (c_int32, [H, c_int32]),
        "gputx_phase_times": (c_int32, [H, POINTER(ctypes.c_double), c_int32, POINTER(c_int64)]),
        "gputx_phase_name": (ctypes.c_char_p, [c_int32]),
        "gputx_batch_create": (c_int32, [H, POINTER(BatchItem), c_int32, POINTER(H)]),
        "gputx_batch_launch": (c_int32, [H, c_void_p]),
        "gputx_batch_destroy": (c_int32, [H]),
        "gputx_serve": (c_int32, [H, POINTER(Trace), POINTER(ServeOpts), c_void_p, c_void_p,
                                  POINTER(ServeBulk), c_int64, POINTER(ServeReport)]),
        "gputx_serve_open": (c_int32, [H, POINTER(ServeOpts), c_int32, c_int64, POINTER(H)]),
        "gputx_serve_submit": (c_int32, [H, c_int64, c_void_p, c_void_p, c_int64, c_void_p,
                                         POINTER(c_int64)]),
        "gputx_serve_poll": (c_int32, [H, c_int64, c_void_p, c_void_p, c_void_p, c_void_p,
                                       POINTER(c_int64)]),
        "gputx_serve_close": (c_int32, [H, POINTER(ServeReport)]),
        "gputx_read_table": (c_int32, [H, c_int32, c_int32, c_int64, c_int64, c_void_p, c_void_p]),
        "gputx_micro_workspace_size": (c_size_t, [c_int64]),
        "gputx_micro_run": (c_int32, [c_int64, c_void_p, c_void_p, c_int32, c_int32, c_int32, c_void_p,
                                      c_size_t, c_int32, c_void_p]),
        "gputx_pool_create": (c_int32, [H, c_int64, c_int32, c_int32, c_int32, c_int64, POINTER(H)]),
        "gputx_pool_add": (c_int32, [H, POINTER(BulkDesc), c_void_p]),
        "gputx_pool_step": (c_int32, [H, c_int32, c_void_p]),
        "gputx_pool_state": (c_int32, [H, POINTER(PoolStats), c_void_p]),
        "gputx_pool_results": (c_int32, [H, c_int64, c_void_p, c_void_p, c_void_p]),
        "gputx_pool_destroy": (c_int32, [H]),
        "gputx_probe_handoff": (c_int32, [c_int32, c_int32, c_int32, POINTER(ctypes.c_double)]),
        "gputx_probe_atomic_add": (c_int32, [c_int32, c_int64, c_int64, POINTER(ctypes.c_double)]),
        "gputx_probe_gather": (c_int32, [c_int32, c_int64, c_int64, POINTER(ctypes.c_double)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()
EXPORTS = ("gputx_default_options", "gputx_create", "gputx_destroy", "gputx_set_options",
           "gputx_load_tables", "gputx_register_types", "gputx_workspace_size",
           "gputx_workspace_size_ops",
           "gputx_execute_bulk", "gputx_row_count", "gputx_set_row_count", "gputx_last_error", "gputx_phase_timing",
           "gputx_phase_times", "gputx_phase_name", "gputx_batch_create", "gputx_batch_launch",
           "gputx_batch_destroy", "gputx_serve", "gputx_probe_handoff", "gputx_probe_atomic_add",
           "gputx_probe_gather", "gputx_execute_bulk_noalloc", "gputx_serve_open",
           "gputx_serve_submit", "gputx_serve_poll", "gputx_serve_close", "gputx_read_table",
           "gputx_micro_workspace_size", "gputx_micro_run", "gputx_execute_bulk_relaxed",
           "gputx_pool_create", "gputx_pool_add", "gputx_pool_step", "gputx_pool_state", "gputx_pool_results", "gputx_pool_destroy")
SCRATCH_BYTES = 64 << 20   # GPUTX_SCRATCH_BYTES: static workspace of gputx_execute_bulk_noalloc


class GputxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gputx error {code}: {msg}")
        self.code = code


def _check(h, rc: int):
    if rc != OK:
        raise GputxError(rc, lib.gputx_last_error(h).decode())


# ---- same-name wrappers ----------------------------------------------------

def gputx_default_options() -> Options:
    o = Options()
    _check(None, lib.gputx_default_options(ctypes.byref(o)))
    return o


def gputx_create(device: int = 0, options: Optional[Options] = None) -> c_void_p:
    h = c_void_p()
    _check(None, lib.gputx_create(device, ctypes.byref(options) if options else None,
                                  ctypes.byref(h)))
    return h


def gputx_destroy(h) -> None:
    _check(h, lib.gputx_destroy(h))


def gputx_set_options(h, options: Options) -> None:
    _check(h, lib.gputx_set_options(h, ctypes.byref(options)))


def gputx_load_tables(h, descs: Sequence[TableDesc]) -> None:
    arr = (TableDesc * len(descs))(*descs)
    _check(h, lib.gputx_load_tables(h, arr, len(descs)))


def gputx_register_types(h, descs: Sequence[TypeDesc]) -> None:
    arr = (TypeDesc * len(descs))(*descs)
    _check(h, lib.gputx_register_types(h, arr, len(descs)))


def gputx_workspace_size(h, n: int) -> int:
    return int(lib.gputx_workspace_size(h, n))


def gputx_workspace_size_ops(h, n: int, max_ops: int) -> int:
    return int(lib.gputx_workspace_size_ops(h, n, max_ops))


def _stream(stream) -> int:
    return (stream or torch.cuda.current_stream()).cuda_stream


def gputx_execute_bulk(h, bulk: BulkDesc, strategy: int, workspace: torch.Tensor,
                       status: torch.Tensor, results: torch.Tensor, stats: torch.Tensor,
                       stream: Optional[torch.cuda.Stream] = None) -> None:
    s = (stream or torch.cuda.current_stream()).cuda_stream
    _check(h, lib.gputx_execute_bulk(h, ctypes.byref(bulk), strategy, workspace.data_ptr(),
                                     workspace.numel() * workspace.element_size(),
                                     status.data_ptr(), results.data_ptr(), results.shape[1],
                                     stats.data_ptr(), s))


def gputx_execute_bulk_relaxed(h, bulk: BulkDesc, strategy: int, workspace: torch.Tensor,
                               status: torch.Tensor, results: torch.Tensor, serial_key: torch.Tensor,
                               stats: torch.Tensor, stream=None) -> None:
    _check(h, lib.gputx_execute_bulk_relaxed(h, ctypes.byref(bulk), strategy, workspace.data_ptr(),
                                             workspace.numel() * workspace.element_size(),
                                             status.data_ptr(), results.data_ptr(), results.shape[1],
                                             serial_key.data_ptr(), stats.data_ptr(), _stream(stream)))


def gputx_execute_bulk_noalloc(h, bulk: BulkDesc, strategy: int, status: torch.Tensor,
                               results: torch.Tensor, stats: torch.Tensor, stream=None) -> None:
    _check(h, lib.gputx_execute_bulk_noalloc(h, ctypes.byref(bulk), strategy, status.data_ptr(),
                                             results.data_ptr(), results.shape[1], stats.data_ptr(),
                                             _stream(stream)))


def gputx_serve_open(h, opts: ServeOpts, n_params: int, pool_capacity: int) -> c_void_p:
    s = c_void_p()
    _check(h, lib.gputx_serve_open(h, ctypes.byref(opts), n_params, pool_capacity, ctypes.byref(s)))
    return s


def gputx_serve_submit(h, s, type_arr: np.ndarray, params: np.ndarray, ts: np.ndarray) -> int:
    """Submit host arrays (type[n] int32, params[P][n] int64, ts[n] int64);
    returns the first ticket."""
    n = int(type_arr.shape[0])
    t = np.ascontiguousarray(type_arr, dtype=np.int32)
    p = np.ascontiguousarray(params, dtype=np.int64)
    x = np.ascontiguousarray(ts, dtype=np.int64)
    first = c_int64()
    _check(h, lib.gputx_serve_submit(s, n, t.ctypes.data, p.ctypes.data, p.shape[1] if p.ndim == 2 else n,
                                     x.ctypes.data, ctypes.byref(first)))
    return first.value


def gputx_serve_poll(h, s, max_n: int, width: int):
    """Up to max_n finished transactions: (tickets, status, results, latency_ns)."""
    tk = np.zeros(max(max_n, 1), np.int64)
    st = np.zeros(max(max_n, 1), np.int32)
    rs = np.zeros((max(max_n, 1), width), np.int64)
    lat = np.zeros(max(max_n, 1), np.int64)
    got = c_int64()
    _check(h, lib.gputx_serve_poll(s, max_n, tk.ctypes.data, st.ctypes.data, rs.ctypes.data,
                                   lat.ctypes.data, ctypes.byref(got)))
    k = got.value
    return tk[:k], st[:k], rs[:k], lat[:k]


def gputx_serve_close(h, s) -> "ServeReport":
    rep = ServeReport()
    _check(h, lib.gputx_serve_close(s, ctypes.byref(rep)))
    return rep


def gputx_read_table(h, table_id: int, col: int, row0: int, n: int, dtype, stream=None) -> np.ndarray:
    out = np.zeros(max(n, 0), dtype=dtype)
    _check(h, lib.gputx_read_table(h, table_id, col, row0, n, out.ctypes.data if n else None,
                                   _stream(stream)))
    return out


def gputx_row_count(h, table_id: int, stream: Optional[torch.cuda.Stream] = None) -> int:
    out = c_int64()
    s = (stream or torch.cuda.current_stream()).cuda_stream
    _check(h, lib.gputx_row_count(h, table_id, ctypes.byref(out), s))
    return out.value


def gputx_set_row_count(h, table_id: int, n: int, stream: Optional[torch.cuda.Stream] = None) -> None:
    s = (stream or torch.cuda.current_stream()).cuda_stream
    _check(h, lib.gputx_set_row_count(h, table_id, n, s))


def gputx_phase_timing(h, enable: bool) -> None:
    _check(h, lib.gputx_phase_timing(h, 1 if enable else 0))


def gputx_phase_name(i: int) -> Optional[str]:
    r = lib.gputx_phase_name(i)
    return r.decode() if r else None


def gputx_phase_times(h) -> tuple:
    """(dict phase -> summed ms, number of bulks summed)."""
    ms = (ctypes.c_double * 32)()
    nb = c_int64()
    k = lib.gputx_phase_times(h, ms, 32, ctypes.byref(nb))
    if k < 0:
        _check(h, k)
    return {gputx_phase_name(i): ms[i] for i in range(k)}, nb.value


def gputx_batch_create(h, items: Sequence[BatchItem]) -> c_void_p:
    arr = (BatchItem * len(items))(*items)
    b = c_void_p()
    _check(h, lib.gputx_batch_create(h, arr, len(items), ctypes.byref(b)))
    return b


def gputx_batch_launch(h, b, stream: Optional[torch.cuda.Stream] = None) -> None:
    s = (stream or torch.cuda.current_stream()).cuda_stream
    _check(h, lib.gputx_batch_launch(b, s))


def gputx_batch_destroy(h, b) -> None:
    _check(h, lib.gputx_batch_destroy(b))


def gputx_serve(h, trace: Trace, opts: ServeOpts, status: torch.Tensor, results: torch.Tensor,
                bulk_capacity: int):
    """Serve a trace; status / results are page-locked host tensors.  Returns
    (report, numpy structured array of per-bulk records)."""
    recs = (ServeBulk * max(bulk_capacity, 1))()
    rep = ServeReport()
    _check(h, lib.gputx_serve(h, ctypes.byref(trace), ctypes.byref(opts), status.data_ptr(),
                              results.data_ptr(), recs, bulk_capacity, ctypes.byref(rep)))
    n = min(rep.n_bulks, bulk_capacity)
    arr = np.ctypeslib.as_array(recs)[:n].copy() if n else np.zeros(0)
    return rep, arr


def gputx_probe_handoff(device: int, hops: int, same_xcd: bool = False) -> float:
    """ns per lock hand-off between two workgroups (see the header)."""
    v = ctypes.c_double()
    _check(None, lib.gputx_probe_handoff(device, hops, 1 if same_xcd else 0, ctypes.byref(v)))
    return v.value


def gputx_probe_atomic_add(device: int, n_addr: int, n_updates: int) -> float:
    """Device atomic adds per second over n_addr addresses."""
    v = ctypes.c_double()
    _check(None, lib.gputx_probe_atomic_add(device, n_addr, n_updates, ctypes.byref(v)))
    return v.value


def gputx_probe_gather(device: int, table_bytes: int, n_gathers: int) -> float:
    """GB/s of 8-byte gathers at uniform random rows of a table_bytes table."""
    v = ctypes.c_double()
    _check(None, lib.gputx_probe_gather(device, table_bytes, n_gathers, ctypes.byref(v)))
    return v.value


def gputx_micro_workspace_size(n: int) -> int:
    return int(lib.gputx_micro_workspace_size(n))


def gputx_micro_run(type_arr: torch.Tensor, tuples: torch.Tensor, n_types: int, x: int, groups: int,
                    workspace: Optional[torch.Tensor] = None, phase: int = 0, stream=None) -> None:
    """Branch-divergence micro benchmark on device arrays (see the header)."""
    n = int(type_arr.shape[0])
    ws_ptr, ws_bytes = (workspace.data_ptr(), workspace.numel()) if workspace is not None else (None, 0)
    _check(None, lib.gputx_micro_run(n, type_arr.data_ptr(), tuples.data_ptr(), n_types, x, groups,
                                     ws_ptr, ws_bytes, phase, _stream(stream)))


def stats_from(t: torch.Tensor) -> BulkStats:
    """Decode a device stats buffer (synchronises via the copy)."""
    raw = t.cpu().numpy().tobytes()
    return BulkStats.from_buffer_copy(raw)


# ---- convenience: one device database -------------------------------------

class Engine:
    """A context with tables copied to the device and types registered.

    ``tables``: name -> object with ``cols``, ``dtypes``, ``n_rows``,
    ``capacity``, ``append``, ``root``, ``root_div`` (as produced by
    ``workloads``); ``types``: objects with ``type_id``, ``proc``,
    ``n_params``, ``n_results``, ``tables`` (role names), ``root_key``.
    """

    def __init__(self, tables: Dict[str, object], types: Sequence[object], device: int = 0,
                 options: Optional[Options] = None, **opt_overrides):
        self.device = torch.device("cuda", device)
        opts = options or gputx_default_options()
        for k, v in opt_overrides.items():
            setattr(opts, k, v)
        self.options = opts
        self.h = gputx_create(device, opts)
        self.table_id: Dict[str, int] = {}
        self.cols: Dict[str, list] = {}
        self.append_tables = {name: bool(t.append) for name, t in tables.items()}
        for i, name in enumerate(tables):
            self.table_id[name] = i
        descs = []
        for name, t in tables.items():
            d = TableDesc()
            d.table_id = self.table_id[name]
            d.n_cols = len(t.cols)
            d.n_rows = t.n_rows
            d.capacity = t.capacity
            d.append_only = 1 if t.append else 0
            d.root_table_id = self.table_id[t.root] if (t.root and t.root_div > 0) else -1
            d.root_div = t.root_div if t.root_div > 0 else 1
            dev_cols = []
            for c, (col, dt) in enumerate(zip(t.cols, t.dtypes)):
                dc = torch.from_numpy(np.ascontiguousarray(col)).to(self.device)
                dev_cols.append(dc)
                d.col_dtype[c] = I64 if dt == "i64" else I32
                d.col_ptr[c] = dc.data_ptr()
            self.cols[name] = dev_cols
            descs.append(d)
        gputx_load_tables(self.h, descs)
        tds = []
        for ty in types:
            td = TypeDesc()
            td.type_id = ty.type_id
            td.proc = PROC[ty.proc]
            td.n_params = ty.n_params
            td.n_results = ty.n_results
            for r in range(MAX_ROLES):
                td.table_ids[r] = self.table_id[ty.tables[r]] if r < len(ty.tables) else -1
            td.root_key = 1 if ty.root_key else 0
            td.single_partition = 1 if getattr(ty, "single_partition", True) else 0
            tds.append(td)
        gputx_register_types(self.h, tds)
        self._ws = None
        self._ws_n = -1

    def set_options(self, **kw):
        for k, v in kw.items():
            setattr(self.options, k, v)
        gputx_set_options(self.h, self.options)
        self._ws_n = -1

    def workspace(self, n: int) -> torch.Tensor:
        if self._ws is None or self._ws_n < n:
            nbytes = gputx_workspace_size(self.h, n)
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self._ws_n = n
        return self._ws

    def bulk_to_device(self, bulk) -> dict:
        # the types the bulk holds (the library sizes PART's layout for them)
        t = np.asarray(bulk.type)
        t = t[(t >= 0) & (t < MAX_TYPES)]
        mask = int(np.bitwise_or.reduce(np.left_shift(1, np.unique(t)).astype(np.uint32))) if t.size else 0
        return dict(type=torch.from_numpy(np.ascontiguousarray(bulk.type)).to(self.device),
                    params=torch.from_numpy(np.ascontiguousarray(bulk.params)).to(self.device),
                    ts=torch.from_numpy(np.ascontiguousarray(bulk.ts)).to(self.device),
                    type_mask=mask)

    @staticmethod
    def bulk_desc(dev: dict, ts_sorted: bool, max_ops: int = 0) -> BulkDesc:
        b = BulkDesc()
        b.max_ops = max_ops
        b.n = dev["type"].shape[0]
        b.type = dev["type"].data_ptr()
        b.params = dev["params"].data_ptr()
        b.n_params = dev["params"].shape[0]
        b.ts = dev["ts"].data_ptr()
        b.ts_sorted = 1 if ts_sorted else 0
        b.type_mask = dev.get("type_mask", 0)
        return b

    def execute(self, dev: dict, strategy: int, width: int, ts_sorted: bool = False,
                status: Optional[torch.Tensor] = None, results: Optional[torch.Tensor] = None,
                stats: Optional[torch.Tensor] = None, stream=None):
        """Launch one bulk (asynchronous).  Returns (status, results, stats) device tensors."""
        n = dev["type"].shape[0]
        if status is None:
            status = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        if results is None:
            results = torch.empty((max(n, 1), width), dtype=torch.int64, device=self.device)
        if stats is None:
            stats = torch.empty(STATS_BYTES, dtype=torch.uint8, device=self.device)
        ws = self.workspace(max(n, 1))
        gputx_execute_bulk(self.h, self.bulk_desc(dev, ts_sorted), strategy, ws, status, results,
                           stats, stream)
        return status, results, stats

    def execute_relaxed(self, dev: dict, strategy: int, width: int, stream=None):
        """One bulk without the timestamp constraint (gputx_execute_bulk_relaxed).
        Returns (status, results, serial_key, stats) device tensors."""
        n = dev["type"].shape[0]
        status = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        results = torch.empty((max(n, 1), width), dtype=torch.int64, device=self.device)
        key = torch.empty(max(n, 1), dtype=torch.int64, device=self.device)
        stats = torch.empty(STATS_BYTES, dtype=torch.uint8, device=self.device)
        ws = self.workspace(max(n, 1))
        gputx_execute_bulk_relaxed(self.h, self.bulk_desc(dev, False), strategy, ws, status, results, key,
                                   stats, stream)
        return status, results, key, stats

    def execute_noalloc(self, dev: dict, strategy: int, width: int, ts_sorted: bool = False,
                        status: Optional[torch.Tensor] = None, results: Optional[torch.Tensor] = None,
                        stats: Optional[torch.Tensor] = None, stream=None):
        """Launch one bulk through gputx_execute_bulk_noalloc (workspace in the
        library's static device array).  Returns (status, results, stats)."""
        n = dev["type"].shape[0]
        if status is None:
            status = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        if results is None:
            results = torch.empty((max(n, 1), width), dtype=torch.int64, device=self.device)
        if stats is None:
            stats = torch.empty(STATS_BYTES, dtype=torch.uint8, device=self.device)
        gputx_execute_bulk_noalloc(self.h, self.bulk_desc(dev, ts_sorted), strategy, status, results,
                                   stats, stream)
        return status, results, stats

    def batch(self, jobs: Sequence[dict]) -> "Batch":
        """jobs: dicts with dev (device bulk), lane, strategy, width and
        optional ts_sorted / max_ops."""
        return Batch(self, jobs)

    def row_count(self, name: str) -> int:
        return gputx_row_count(self.h, self.table_id[name])

    def truncate_appends(self, n: int = 0) -> None:
        """Set every append-only table's row count to n (default: empty)."""
        for name, tid in self.table_id.items():
            if self.append_tables.get(name):
                gputx_set_row_count(self.h, tid, n)

    def table_host(self, name: str) -> list:
        return [c.cpu().numpy() for c in self.cols[name]]

    def close(self):
        if self.h:
            gputx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many bulks captured into one HIP graph (``gputx_batch_create``); every
    job gets its own workspace and output buffers."""

    def __init__(self, eng: Engine, jobs: Sequence[dict]):
        self.eng = eng
        self.jobs = list(jobs)
        self.outputs = []
        items = []
        for j in self.jobs:
            dev = j["dev"]
            n = int(dev["type"].shape[0])
            width = int(j["width"])
            max_ops = int(j.get("max_ops", 0))
            ws = torch.empty(gputx_workspace_size_ops(eng.h, max(n, 1), max_ops), dtype=torch.uint8,
                             device=eng.device)
            st = torch.empty(max(n, 1), dtype=torch.int32, device=eng.device)
            res = torch.empty((max(n, 1), width), dtype=torch.int64, device=eng.device)
            stats = torch.empty(STATS_BYTES, dtype=torch.uint8, device=eng.device)
            it = BatchItem()
            it.bulk = Engine.bulk_desc(dev, bool(j.get("ts_sorted", True)), max_ops)
            it.strategy = int(j["strategy"])
            it.lane = int(j["lane"])
            it.workspace = ws.data_ptr()
            it.ws_bytes = ws.numel()
            it.status_out = st.data_ptr()
            it.results_out = res.data_ptr()
            it.width = width
            it.stats = stats.data_ptr()
            it.grid_blocks = int(j.get("grid_blocks", 0))
            it.kset_narrow = int(j.get("kset_narrow", 0))
            items.append(it)
            self.outputs.append(dict(ws=ws, status=st, results=res, stats=stats, n=n))
        self.b = gputx_batch_create(eng.h, items)

    def launch(self, stream=None) -> None:
        gputx_batch_launch(self.eng.h, self.b, stream)

    def stats(self, k: int) -> BulkStats:
        return stats_from(self.outputs[k]["stats"])

    def close(self) -> None:
        if self.b:
            gputx_batch_destroy(self.eng.h, self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pool:
    """K-SET over a standing pool (gputx_pool_*): add bulks in timestamp
    order, run 0-sets, fetch results in sequence order."""

    def __init__(self, eng: "Engine", capacity: int, n_params: int, width: int, max_ops: int = 0,
                 max_add: int = 1 << 16):
        self.eng = eng
        self.width = width
        self.p = c_void_p()
        _check(eng.h, lib.gputx_pool_create(eng.h, capacity, n_params, width, max_ops, max_add,
                                            ctypes.byref(self.p)))
        self._keep = []

    def add(self, dev: dict, ts_sorted: bool = False, stream=None) -> None:
        self._keep.append(dev)   # the bulk's arrays must live until the add has run
        _check(self.eng.h, lib.gputx_pool_add(self.p, ctypes.byref(Engine.bulk_desc(dev, ts_sorted)),
                                              _stream(stream)))

    def step(self, waves: int = 1, stream=None) -> None:
        _check(self.eng.h, lib.gputx_pool_step(self.p, waves, _stream(stream)))

    def state(self, stream=None) -> PoolStats:
        st = PoolStats()
        _check(self.eng.h, lib.gputx_pool_state(self.p, ctypes.byref(st), _stream(stream)))
        self._keep.clear()       # synchronised: earlier adds have run
        return st

    def results(self, n: int, stream=None):
        status = np.zeros(max(n, 1), np.int32)
        res = np.zeros((max(n, 1), self.width), np.int64)
        _check(self.eng.h, lib.gputx_pool_results(self.p, n, status.ctypes.data, res.ctypes.data,
                                                  _stream(stream)))
        return status[:n], res[:n]

    def close(self) -> None:
        if self.p:
            lib.gputx_pool_destroy(self.p)
            self.p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
