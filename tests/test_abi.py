"""The C-ABI library loads and exports what include/gputx.h declares; the
ctypes layouts match the header (checked by compiling it with gcc).  CPU only:
no compute call is made."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gputx.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(gputx_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    from paper_1103_3105_amd import gputx
    names = _declared()
    assert len(names) >= 10
    lib = ctypes.CDLL(gputx.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(gputx.EXPORTS) == set(names)


def test_struct_layout_matches_header(tmp_path):
    from paper_1103_3105_amd import gputx
    prog = tmp_path / "layout.c"
    prog.write_text('#include <stdio.h>\n#include "gputx.h"\n#include <stddef.h>\nint main(void){\n'
                    'printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", '
                    'sizeof(gputx_options), '
                    'sizeof(gputx_table_desc), sizeof(gputx_type_desc), sizeof(gputx_bulk), '
                    'sizeof(gputx_bulk_stats), offsetof(gputx_table_desc, col_ptr), '
                    'offsetof(gputx_bulk, ts), offsetof(gputx_bulk_stats, appended), '
                    'sizeof(gputx_batch_item), offsetof(gputx_batch_item, stats), '
                    'sizeof(gputx_trace), sizeof(gputx_serve_opts), sizeof(gputx_serve_bulk), '
                    'sizeof(gputx_serve_report));\n'
                    'return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.dirname(HEADER), str(prog), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(gputx.Options), ctypes.sizeof(gputx.TableDesc),
            ctypes.sizeof(gputx.TypeDesc), ctypes.sizeof(gputx.BulkDesc),
            ctypes.sizeof(gputx.BulkStats), gputx.TableDesc.col_ptr.offset,
            gputx.BulkDesc.ts.offset, gputx.BulkStats.appended.offset,
            ctypes.sizeof(gputx.BatchItem), gputx.BatchItem.stats.offset,
            ctypes.sizeof(gputx.Trace), ctypes.sizeof(gputx.ServeOpts),
            ctypes.sizeof(gputx.ServeBulk), ctypes.sizeof(gputx.ServeReport)]
    assert got == want


def test_enums_match_header():
    from paper_1103_3105_amd import gputx
    src = open(HEADER).read()
    for name, val in gputx.PROC.items():
        assert re.search(rf"GPUTX_{name}\s*=\s*{val}\b", src), name
    for name, val in gputx.STRATEGY.items():
        assert re.search(rf"GPUTX_{name}\s*=\s*{val}\b", src), name


def test_errors_without_gpu_are_reported_not_thrown():
    from paper_1103_3105_amd import gputx
    # a null handle is rejected by the ABI itself, before any device call
    assert gputx.lib.gputx_destroy(None) == gputx.E_ARG
    assert gputx.lib.gputx_workspace_size(None, 10) == 0
    o = gputx.gputx_default_options()
    assert o.part_size >= 1 and o.spin_limit_ms > 0
