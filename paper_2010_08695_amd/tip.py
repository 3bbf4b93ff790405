"""ctypes binding of libtip (include/tip.h).

Argument marshalling only: every step of counting and decomposition runs in
the HIP kernels of libtip.so.  If the library has not been built, loading
raises instead of falling back to anything else.

Graph arguments are any object with ``n_u``, ``n_v``, ``eu``, ``ev``
(e.g. ``graphgen.Graph``); ``eu``/``ev`` are int32 arrays of 0-based ids.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtip.so")

TIP_OK, TIP_EINVAL, TIP_ENOMEM, TIP_EDEVICE, TIP_EOVERFLOW, TIP_EBUSY = 0, -1, -2, -3, -4, -5
TIP_FLAG_TIME_KERNELS = 1
TIP_FLAG_NO_GRAPH = 2
TIP_FLAG_BATCH_PLAIN = 4
TIP_FLAG_NO_COMPACT = 8
TIP_FLAG_OPTS_PER_GRAPH = 16
TIP_FLAG_BATCH_STREAMS = 32
TIP_FLAG_FD_DGM = 64
TIP_FLAG_DGM_PAPER = 128
TIP_FLAG_FD_WALK = 256
SIDE_U, SIDE_V = 0, 1
STATUS_NAMES = {0: "TIP_OK", -1: "TIP_EINVAL", -2: "TIP_ENOMEM", -3: "TIP_EDEVICE",
                -4: "TIP_EOVERFLOW", -5: "TIP_EBUSY"}

# Every symbol declared in include/tip.h.
EXPORTS = ["tip_count_butterflies", "tip_decompose", "tip_decompose_ex", "tip_decompose_batch",
           "tip_workspace_size", "tip_decompose_async", "tip_decompose_noalloc", "tip_count_edge_butterflies",
           "tip_wing_decompose", "tip_ktips", "tip_last_error", "tip_device_count"]


class TipError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


class Edges(ctypes.Structure):
    _fields_ = [("n_u", ctypes.c_int32), ("n_v", ctypes.c_int32), ("m", ctypes.c_int64),
                ("eu", ctypes.c_void_p), ("ev", ctypes.c_void_p)]


class Opts(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int32), ("flags", ctypes.c_int32), ("tune", ctypes.c_int32 * 8)]


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("wedges_count", "wedges_cd", "wedges_fd", "pair_updates", "rounds", "subsets",
                 "fd_levels", "spills", "skipped", "m_unique",
                 "peel_launches", "peel_wedges", "peel_edges", "peel_pairs")] + \
               [(n, ctypes.c_double) for n in
                ("peel_ms", "t_ingest_ms", "t_count_ms", "t_cd_ms", "t_fd_ms", "t_total_ms")] + \
               [("huc_rounds", ctypes.c_int64), ("fd_huc_steps", ctypes.c_int64), ("compactions", ctypes.c_int64),
                ("fd_pair_entries", ctypes.c_int64), ("fd_pair_subsets", ctypes.c_int64)]

    def to_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_lock = threading.Lock()
_lib = None


def _bind_hip_runtime():
    # One HIP runtime per process: when PyTorch is installed, load it first so
    # that libtip binds to the HIP runtime torch already uses (same soname)
    # instead of a second copy that would make torch's device init fail.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def load(path: str | None = None) -> ctypes.CDLL:
    """Loads libtip.so; raises FileNotFoundError if it has not been built."""
    global _lib
    _bind_hip_runtime()
    with _lock:
        if _lib is not None and path is None:
            return _lib
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise FileNotFoundError(
                f"{p} is missing: build it with `python -m paper_2010_08695_amd.build` "
                "(there is no fallback implementation)")
        lib = ctypes.CDLL(p)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        lib.tip_count_butterflies.argtypes = [ctypes.POINTER(Edges), vp, vp, vp]
        lib.tip_decompose.argtypes = [ctypes.POINTER(Edges), i32, vp, ctypes.POINTER(Opts), ctypes.POINTER(Stats)]
        lib.tip_decompose_ex.argtypes = [ctypes.POINTER(Edges), i32, vp, ctypes.POINTER(Opts),
                                         ctypes.POINTER(Stats), vp, vp, vp, vp]
        lib.tip_decompose_batch.argtypes = [i32, ctypes.POINTER(Edges), vp, vp, ctypes.POINTER(Opts),
                                            ctypes.POINTER(Stats)]
        lib.tip_workspace_size.argtypes = [i32, i32, i64, i32, ctypes.POINTER(Opts),
                                           ctypes.POINTER(ctypes.c_size_t)]
        lib.tip_decompose_async.argtypes = [vp, vp, i32, i32, i64, i32, vp, vp, ctypes.c_size_t, vp,
                                            ctypes.POINTER(Opts), ctypes.POINTER(Stats)]
        lib.tip_decompose_noalloc.argtypes = [vp, vp, i32, i32, i64, i32, vp, vp, ctypes.POINTER(Opts),
                                              ctypes.POINTER(Stats)]
        lib.tip_count_edge_butterflies.argtypes = [ctypes.POINTER(Edges), vp, vp]
        lib.tip_wing_decompose.argtypes = [ctypes.POINTER(Edges), vp, ctypes.POINTER(Opts), ctypes.POINTER(Stats)]
        lib.tip_ktips.argtypes = [ctypes.POINTER(Edges), i32, vp, i64, vp]
        for name in EXPORTS[:10]:
            getattr(lib, name).restype = ctypes.c_int32
        lib.tip_last_error.argtypes = []
        lib.tip_last_error.restype = ctypes.c_char_p
        lib.tip_device_count.argtypes = []
        lib.tip_device_count.restype = ctypes.c_int32
        if path is None:
            _lib = lib
        return lib


def device_available() -> bool:
    return load().tip_device_count() > 0


def _check(lib, rc: int):
    if rc != TIP_OK:
        raise TipError(rc, (lib.tip_last_error() or b"").decode())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _edges(g) -> tuple[Edges, tuple]:
    eu = np.ascontiguousarray(g.eu, dtype=np.int32)
    ev = np.ascontiguousarray(g.ev, dtype=np.int32)
    if eu.shape != ev.shape:
        raise ValueError("eu and ev differ in length")
    e = Edges(int(g.n_u), int(g.n_v), int(eu.shape[0]), _ptr(eu), _ptr(ev))
    return e, (eu, ev)


def _opts(P: int = 0, flags: int = 0, dense_threshold: int = 0, tune=None) -> Opts:
    o = Opts()
    o.P = int(P)
    o.flags = int(flags)
    for i, t in enumerate(tune or ()):
        o.tune[i] = int(t)
    if dense_threshold:
        o.tune[0] = int(dense_threshold)
    return o


def count_butterflies(g):
    """Per-vertex butterfly counts: (bfly_u int64[n_u], bfly_v int64[n_v], total)."""
    lib = load()
    e, keep = _edges(g)
    bu = np.zeros(g.n_u, np.int64)
    bv = np.zeros(g.n_v, np.int64)
    tot = np.zeros(1, np.int64)
    _check(lib, lib.tip_count_butterflies(ctypes.byref(e), _ptr(bu), _ptr(bv), _ptr(tot)))
    return bu, bv, int(tot[0])


def decompose(g, side: int = SIDE_U, P: int = 0, with_stats: bool = False, flags: int = 0,
              dense_threshold: int = 0, tune=None):
    """Tip numbers int64[n_side] of ``side``; with_stats adds a stats dict.
    tune: tip_opts.tune values (0 = library default); dense_threshold is
    tune[0]."""
    lib = load()
    e, keep = _edges(g)
    n = g.n_u if side == SIDE_U else g.n_v
    theta = np.zeros(max(n, 0), np.int64)
    st = Stats()
    o = _opts(P, flags, dense_threshold, tune)
    _check(lib, lib.tip_decompose(ctypes.byref(e), int(side), _ptr(theta), ctypes.byref(o), ctypes.byref(st)))
    return (theta, st.to_dict()) if with_stats else theta


def decompose_ex(g, side: int = SIDE_U, P: int = 0, flags: int = 0, tune=None) -> dict:
    """Tip numbers plus the coarse-grained state (subsets, initial supports, bounds)."""
    lib = load()
    e, keep = _edges(g)
    n = g.n_u if side == SIDE_U else g.n_v
    Pe = P if P > 0 else 150
    theta = np.zeros(n, np.int64)
    subset = np.zeros(n, np.int32)
    init = np.zeros(n, np.int64)
    bounds = np.zeros(Pe + 2, np.int64)
    ns = np.zeros(1, np.int32)
    st = Stats()
    o = _opts(P, flags, 0, tune)
    _check(lib, lib.tip_decompose_ex(ctypes.byref(e), int(side), _ptr(theta), ctypes.byref(o),
                                     ctypes.byref(st), _ptr(subset), _ptr(init), _ptr(bounds), _ptr(ns)))
    k = int(ns[0])
    return {"theta": theta, "subset": subset, "init": init, "bounds": bounds[:k + 1],
            "n_subsets": k, "stats": st.to_dict()}


def batch_opts(n: int, P: int, flags: int, tunes) -> ctypes.Array:
    """tip_opts[n] for tip_decompose_batch with TIP_FLAG_OPTS_PER_GRAPH:
    graph k gets tunes[k] (None = the library defaults)."""
    if len(tunes) != n:
        raise ValueError("one tune entry per graph")
    arr = (Opts * max(n, 1))()
    for k in range(n):
        arr[k] = _opts(P, flags | TIP_FLAG_OPTS_PER_GRAPH, 0, tunes[k])
    return arr


def decompose_batch(graphs, sides=None, P: int = 0, with_stats: bool = False, flags: int = 0, tunes=None):
    """Tip numbers of many graphs in one call (batched form unless flags has
    TIP_FLAG_BATCH_PLAIN).  tunes: None, or one tip_opts.tune list (or None
    for the defaults) per graph, passed with TIP_FLAG_OPTS_PER_GRAPH."""
    lib = load()
    n = len(graphs)
    sides = [SIDE_U] * n if sides is None else list(sides)
    es = (Edges * max(n, 1))()
    keep, thetas = [], []
    for k, g in enumerate(graphs):
        e, kp = _edges(g)
        es[k] = e
        keep.append(kp)
        thetas.append(np.zeros(g.n_u if sides[k] == SIDE_U else g.n_v, np.int64))
    sides_a = np.ascontiguousarray(sides, dtype=np.int32)
    ptrs = (ctypes.c_void_p * max(n, 1))(*[t.ctypes.data for t in thetas])
    sts = (Stats * max(n, 1))()
    popt = batch_opts(n, P, flags, tunes) if tunes is not None else ctypes.byref(_opts(P, flags))
    _check(lib, lib.tip_decompose_batch(n, es, _ptr(sides_a), ctypes.cast(ptrs, ctypes.c_void_p), popt, sts))
    if with_stats:
        return thetas, [sts[k].to_dict() for k in range(n)]
    return thetas


def workspace_size(n_u: int, n_v: int, m: int, side: int = SIDE_U, P: int = 0, flags: int = 0) -> int:
    lib = load()
    out = ctypes.c_size_t(0)
    o = _opts(P, flags)
    _check(lib, lib.tip_workspace_size(int(n_u), int(n_v), int(m), int(side), ctypes.byref(o), ctypes.byref(out)))
    return int(out.value)


def decompose_async(d_eu, d_ev, n_u: int, n_v: int, side: int, d_theta, workspace, stream=None,
                    P: int = 0, flags: int = 0, dense_threshold: int = 0, tune=None) -> dict:
    """Device-resident decomposition.  d_eu/d_ev/d_theta/workspace are torch
    CUDA(HIP) tensors (only their device pointers are passed); stream is a
    torch.cuda.Stream or None for the current stream.  Returns the stats."""
    lib = load()
    m = int(d_eu.numel())
    if int(d_ev.numel()) != m:
        raise ValueError("eu and ev differ in length")
    s = None
    if stream is not None:
        s = stream.cuda_stream
    else:
        import torch
        s = torch.cuda.current_stream().cuda_stream
    st = Stats()
    o = _opts(P, flags, dense_threshold, tune)
    _check(lib, lib.tip_decompose_async(
        ctypes.c_void_p(d_eu.data_ptr()), ctypes.c_void_p(d_ev.data_ptr()), int(n_u), int(n_v), m, int(side),
        ctypes.c_void_p(d_theta.data_ptr()), ctypes.c_void_p(workspace.data_ptr()),
        int(workspace.numel() * workspace.element_size()), ctypes.c_void_p(s), ctypes.byref(o),
        ctypes.byref(st)))
    return st.to_dict()


NOALLOC_SCRATCH_BYTES = 512 << 20


def decompose_noalloc(d_eu, d_ev, n_u: int, n_v: int, side: int, d_theta, stream=None, P: int = 0,
                      flags: int = 0, tune=None) -> dict:
    """tip_decompose_noalloc: like decompose_async with TIP_FLAG_FD_WALK, with
    the library's static device scratch instead of a workspace (graphs whose
    workspace_size(..., flags=TIP_FLAG_FD_WALK) exceeds NOALLOC_SCRATCH_BYTES
    are refused with TIP_ENOMEM).  Returns the stats."""
    lib = load()
    m = int(d_eu.numel())
    if int(d_ev.numel()) != m:
        raise ValueError("eu and ev differ in length")
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    st = Stats()
    o = _opts(P, flags, 0, tune)
    _check(lib, lib.tip_decompose_noalloc(
        ctypes.c_void_p(d_eu.data_ptr()), ctypes.c_void_p(d_ev.data_ptr()), int(n_u), int(n_v), m, int(side),
        ctypes.c_void_p(d_theta.data_ptr()), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(o),
        ctypes.byref(st)))
    return st.to_dict()


def count_edge_butterflies(g):
    """Butterflies containing each input edge: (int64[m], total)."""
    lib = load()
    e, keep = _edges(g)
    out = np.zeros(max(g.m, 1), np.int64)
    tot = np.zeros(1, np.int64)
    _check(lib, lib.tip_count_edge_butterflies(ctypes.byref(e), _ptr(out), _ptr(tot)))
    return out[:g.m], int(tot[0])


def wing_decompose(g, with_stats: bool = False):
    """Wing number of each input edge: int64[m] (and the stats)."""
    lib = load()
    e, keep = _edges(g)
    out = np.zeros(max(g.m, 1), np.int64)
    st = Stats()
    _check(lib, lib.tip_wing_decompose(ctypes.byref(e), _ptr(out), None, ctypes.byref(st)))
    return (out[:g.m], st.to_dict()) if with_stats else out[:g.m]


def ktips(g, side: int, theta, k: int):
    """k-tips of one side: int32 label per vertex (smallest id of its k-tip,
    -1 when theta < k)."""
    lib = load()
    e, keep = _edges(g)
    n = g.n_u if side == SIDE_U else g.n_v
    theta = np.ascontiguousarray(theta, dtype=np.int64)
    if theta.shape != (n,):
        raise ValueError("one tip number per vertex of the side")
    comp = np.zeros(max(n, 1), np.int32)
    _check(lib, lib.tip_ktips(ctypes.byref(e), int(side), _ptr(theta), int(k), _ptr(comp)))
    return comp[:n]
