"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, struct layouts agree, and argument errors are reported as
TIP_EINVAL on the host before any device work."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

from paper_2010_08695_amd import tip

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tip.h")


@pytest.fixture(scope="module")
def lib():
    return tip.load()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tip_[a-z_]+)\s*\(", src)))


def test_header_declares_the_binding_exports():
    assert declared_functions() == sorted(tip.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(FileNotFoundError):
        tip.load(str(tmp_path / "libtip.so"))


def test_struct_sizes():
    assert ctypes.sizeof(tip.Edges) == 4 + 4 + 8 + 8 + 8
    assert ctypes.sizeof(tip.Opts) == 4 * 10
    assert ctypes.sizeof(tip.Stats) == 14 * 8 + 6 * 8 + 5 * 8


def _header_without_comments():
    return re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)


def test_binding_constants_match_the_header():
    """Every TIP_FLAG_* and status value the header defines has the same value
    in the binding, and the binding defines no flag the header lacks."""
    src = _header_without_comments()
    flags = {n: int(v) for n, v in re.findall(r"#define\s+(TIP_FLAG_[A-Z_]+)\s+(\d+)", src)}
    assert flags and flags == {n: getattr(tip, n) for n in dir(tip) if n.startswith("TIP_FLAG_")}
    assert len(set(flags.values())) == len(flags)
    assert all(v & (v - 1) == 0 for v in flags.values())   # one bit each
    status = dict(re.findall(r"\b(TIP_[A-Z]+)\s*=\s*(-?\d+)", src))
    for name in ("TIP_OK", "TIP_EINVAL", "TIP_ENOMEM", "TIP_EDEVICE", "TIP_EOVERFLOW", "TIP_EBUSY"):
        assert int(status[name]) == getattr(tip, name), name


def test_stats_fields_match_the_header():
    """tip.Stats lists tip_stats' fields in the header's order with the same
    C types, so every field lands at its offset."""
    body = re.search(r"typedef struct \{([^{}]*)\} tip_stats;", _header_without_comments()).group(1)
    fields = []
    for decl in filter(None, (d.strip() for d in body.split(";"))):
        ctype, names = decl.split(None, 1)
        fields += [(n.strip(), ctype) for n in names.split(",")]
    want = {"int64_t": ctypes.c_int64, "double": ctypes.c_double}
    assert [(n, want[t]) for n, t in fields] == list(tip.Stats._fields_)


def _edges(n_u, n_v, eu, ev, m=None):
    eu = np.asarray(eu, np.int32)
    ev = np.asarray(ev, np.int32)
    e = tip.Edges(n_u, n_v, len(eu) if m is None else m, eu.ctypes.data_as(ctypes.c_void_p),
                  ev.ctypes.data_as(ctypes.c_void_p))
    return e, (eu, ev)


def _expect_einval(lib, rc):
    assert rc == tip.TIP_EINVAL, rc
    assert lib.tip_last_error()  # a message is set


def test_count_rejects_bad_arguments(lib):
    out = np.zeros(8, np.int64)
    p = out.ctypes.data_as(ctypes.c_void_p)
    _expect_einval(lib, lib.tip_count_butterflies(None, p, p, p))
    e, k = _edges(2, 2, [0, 2], [0, 1])          # U id out of range
    _expect_einval(lib, lib.tip_count_butterflies(ctypes.byref(e), p, p, p))
    e, k = _edges(2, 2, [0, 1], [0, -1])         # negative V id
    _expect_einval(lib, lib.tip_count_butterflies(ctypes.byref(e), p, p, p))
    e, k = _edges(-1, 2, [], [])
    _expect_einval(lib, lib.tip_count_butterflies(ctypes.byref(e), p, p, p))
    e = tip.Edges(2, 2, 3, None, None)           # m > 0 with NULL arrays
    _expect_einval(lib, lib.tip_count_butterflies(ctypes.byref(e), p, p, p))
    e = tip.Edges(2, 2, -1, None, None)
    _expect_einval(lib, lib.tip_count_butterflies(ctypes.byref(e), p, p, p))
    e = tip.Edges(2, 2, 2**31, None, None)       # too many edges
    _expect_einval(lib, lib.tip_count_butterflies(ctypes.byref(e), p, p, p))


def test_decompose_rejects_bad_arguments(lib):
    theta = np.full(4, 7, np.int64)
    tp = theta.ctypes.data_as(ctypes.c_void_p)
    e, k = _edges(3, 3, [0, 1], [1, 2])
    _expect_einval(lib, lib.tip_decompose(ctypes.byref(e), 2, tp, None, None))
    _expect_einval(lib, lib.tip_decompose(ctypes.byref(e), -1, tp, None, None))
    _expect_einval(lib, lib.tip_decompose(ctypes.byref(e), 0, None, None, None))
    o = tip.Opts()
    o.P = -3
    _expect_einval(lib, lib.tip_decompose(ctypes.byref(e), 0, tp, ctypes.byref(o), None))
    o.P = 70000
    _expect_einval(lib, lib.tip_decompose(ctypes.byref(e), 0, tp, ctypes.byref(o), None))
    o = tip.Opts()
    o.flags = 512                                 # no such flag
    _expect_einval(lib, lib.tip_decompose(ctypes.byref(e), 0, tp, ctypes.byref(o), None))
    o = tip.Opts()
    o.tune[1] = -1
    _expect_einval(lib, lib.tip_decompose(ctypes.byref(e), 0, tp, ctypes.byref(o), None))
    o = tip.Opts()
    o.tune[2] = -5
    _expect_einval(lib, lib.tip_decompose(ctypes.byref(e), 0, tp, ctypes.byref(o), None))
    o = tip.Opts()
    o.tune[3] = -1                                # HUC threshold must be >= 0
    _expect_einval(lib, lib.tip_decompose(ctypes.byref(e), 0, tp, ctypes.byref(o), None))
    o = tip.Opts()
    o.tune[7] = -2                                # fine-grained HUC threshold must be >= 0
    _expect_einval(lib, lib.tip_decompose(ctypes.byref(e), 0, tp, ctypes.byref(o), None))
    o = tip.Opts()
    o.tune[4] = 2**20 + 1                         # help-board claim too large
    _expect_einval(lib, lib.tip_decompose(ctypes.byref(e), 0, tp, ctypes.byref(o), None))
    o = tip.Opts()
    o.tune[6] = -1
    _expect_einval(lib, lib.tip_decompose(ctypes.byref(e), 0, tp, ctypes.byref(o), None))
    o = tip.Opts()
    o.flags = tip.TIP_FLAG_OPTS_PER_GRAPH         # batch-only flag
    _expect_einval(lib, lib.tip_decompose(ctypes.byref(e), 0, tp, ctypes.byref(o), None))
    e, k = _edges(3, 3, [0, 5], [1, 2])
    _expect_einval(lib, lib.tip_decompose(ctypes.byref(e), 0, tp, None, None))
    # outputs untouched by argument errors
    assert (theta == 7).all()


def test_batch_and_workspace_reject_bad_arguments(lib):
    _expect_einval(lib, lib.tip_decompose_batch(-1, None, None, None, None, None))
    _expect_einval(lib, lib.tip_decompose_batch(2, None, None, None, None, None))
    es = (tip.Edges * 1)()
    e, k = _edges(2, 2, [0, 3], [0, 0])
    es[0] = e
    sides = np.zeros(1, np.int32)
    th = np.zeros(2, np.int64)
    ptrs = (ctypes.c_void_p * 1)(th.ctypes.data)
    _expect_einval(lib, lib.tip_decompose_batch(1, es, sides.ctypes.data_as(ctypes.c_void_p),
                                                ctypes.cast(ptrs, ctypes.c_void_p), None, None))
    # per-graph options whose flags differ between graphs
    es2 = (tip.Edges * 2)()
    e0, k0 = _edges(2, 2, [0, 1], [0, 1])
    es2[0] = es2[1] = e0
    th2 = [np.zeros(2, np.int64), np.zeros(2, np.int64)]
    ptrs2 = (ctypes.c_void_p * 2)(th2[0].ctypes.data, th2[1].ctypes.data)
    opts = tip.batch_opts(2, 0, 0, [None, None])
    opts[1].flags = tip.TIP_FLAG_OPTS_PER_GRAPH | tip.TIP_FLAG_NO_COMPACT
    _expect_einval(lib, lib.tip_decompose_batch(2, es2, np.zeros(2, np.int32).ctypes.data_as(ctypes.c_void_p),
                                                ctypes.cast(ptrs2, ctypes.c_void_p), opts, None))
    out = ctypes.c_size_t(0)
    _expect_einval(lib, lib.tip_workspace_size(2, 2, 4, 0, None, None))
    _expect_einval(lib, lib.tip_workspace_size(2, 2, -4, 0, None, ctypes.byref(out)))
    _expect_einval(lib, lib.tip_workspace_size(2, 2, 4, 3, None, ctypes.byref(out)))


def test_async_rejects_bad_arguments(lib):
    _expect_einval(lib, lib.tip_decompose_async(None, None, 2, 2, 4, 0, None, None, 0, None, None, None))
    _expect_einval(lib, lib.tip_decompose_async(None, None, 2, 2, 0, 5, None, None, 0, None, None, None))
    _expect_einval(lib, lib.tip_decompose_async(None, None, -2, 2, 0, 0, None, None, 0, None, None, None))


def test_last_error_is_per_call(lib):
    e, k = _edges(2, 2, [0, 9], [0, 0])
    assert lib.tip_count_butterflies(ctypes.byref(e), None, None, None) == tip.TIP_EINVAL
    assert b"out of range" in lib.tip_last_error()
