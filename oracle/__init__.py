"""CPU oracle for butterfly counting and tip decomposition.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use this package to check and time the GPU path.  The
product library never imports it.

* ``count(g)``            per-vertex butterfly counts of both sides + total
                          (plain 2-hop definition, notation table of the paper)
* ``count_side(g, side)`` per-vertex butterfly counts of one side only
* ``bup(g, side)``        tip numbers by sequential bottom-up peeling (Alg. 2)
* ``support_in(g, side, member, query)``
                          f_x(S) for sampled vertices, for property checks
* ``support_levels(g, side, theta, query)``
                          f_x(S) for S = the side, theta >= theta_x and
                          theta > theta_x, from one build of the adjacency
* ``canonical_edges(g)``  the simple edge list (duplicates merged, sorted by
                          (u, v)); the edge order of the three calls below
* ``edge_count(g)``       butterflies containing each canonical edge
* ``wing(g)``             wing numbers by sequential bottom-up edge peeling
* ``ktip(g, side, theta, k)``
                          k-tips (Def. 1): butterfly-connected components of
                          {theta >= k}, labelled by their smallest vertex id
* ``brute``               exponential brute force for tiny graphs
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "tip_oracle.cpp"), os.path.join(_HERE, "wing_oracle.cpp")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with the host C++ compiler; returns the .so path."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < max(os.path.getmtime(s) for s in _SRCS):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC",
                               *_SRCS, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load(path: str | None = None):
    global _lib
    with _lock:
        if path is not None:
            lib = ctypes.CDLL(path)
        elif _lib is None:
            lib = _lib = ctypes.CDLL(build())
        else:
            return _lib
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    p = ctypes.c_void_p
    lib.oracle_count.argtypes = [i32, i32, i64, p, p, p, p, p]
    lib.oracle_count.restype = ctypes.c_int
    lib.oracle_count_side.argtypes = [i32, i32, i64, p, p, i32, p]
    lib.oracle_count_side.restype = ctypes.c_int
    lib.oracle_bup.argtypes = [i32, i32, i64, p, p, i32, p, p, p]
    lib.oracle_bup.restype = ctypes.c_int
    lib.oracle_support_in.argtypes = [i32, i32, i64, p, p, i32, p, p, i64, p]
    lib.oracle_support_in.restype = ctypes.c_int
    lib.oracle_support_levels.argtypes = [i32, i32, i64, p, p, i32, p, p, i64, p]
    lib.oracle_support_levels.restype = ctypes.c_int
    lib.oracle_canonical_edges.argtypes = [i32, i32, i64, p, p, p, p, p]
    lib.oracle_canonical_edges.restype = ctypes.c_int
    lib.oracle_edge_count.argtypes = [i32, i32, i64, p, p, p]
    lib.oracle_edge_count.restype = ctypes.c_int
    lib.oracle_wing.argtypes = [i32, i32, i64, p, p, p, p, p]
    lib.oracle_wing.restype = ctypes.c_int
    lib.oracle_ktip.argtypes = [i32, i32, i64, p, p, i32, p, i64, p]
    lib.oracle_ktip.restype = ctypes.c_int
    return lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _edges(g):
    eu = np.ascontiguousarray(g.eu, dtype=np.int32)
    ev = np.ascontiguousarray(g.ev, dtype=np.int32)
    return eu, ev


def count(g, lib=None):
    """Returns (bfly_u int64[n_u], bfly_v int64[n_v], total int)."""
    lib = lib or _load()
    eu, ev = _edges(g)
    bu = np.zeros(g.n_u, np.int64)
    bv = np.zeros(g.n_v, np.int64)
    tot = np.zeros(1, np.int64)
    rc = lib.oracle_count(g.n_u, g.n_v, g.m, _ptr(eu), _ptr(ev), _ptr(bu), _ptr(bv), _ptr(tot))
    if rc != 0:
        raise ValueError("oracle_count: invalid graph")
    return bu, bv, int(tot[0])


def count_side(g, side: int, lib=None) -> np.ndarray:
    """Per-vertex butterfly counts of one side: int64[n_u] or int64[n_v]."""
    lib = lib or _load()
    eu, ev = _edges(g)
    out = np.zeros(g.n_u if side == 0 else g.n_v, np.int64)
    rc = lib.oracle_count_side(g.n_u, g.n_v, g.m, _ptr(eu), _ptr(ev), side, _ptr(out))
    if rc != 0:
        raise ValueError("oracle_count_side: invalid graph or side")
    return out


def bup(g, side: int = 0, lib=None):
    """Returns (theta int64[n_side], peel order int32[n_side], wedges int)."""
    lib = lib or _load()
    eu, ev = _edges(g)
    n = g.n_u if side == 0 else g.n_v
    theta = np.zeros(n, np.int64)
    order = np.zeros(n, np.int32)
    wedges = np.zeros(1, np.int64)
    rc = lib.oracle_bup(g.n_u, g.n_v, g.m, _ptr(eu), _ptr(ev), side, _ptr(theta),
                        _ptr(order), _ptr(wedges))
    if rc != 0:
        raise ValueError("oracle_bup: invalid graph or side")
    return theta, order, int(wedges[0])


def support_in(g, side: int, member: np.ndarray, query: np.ndarray, lib=None) -> np.ndarray:
    """f_x(S) for each x in ``query``; ``member`` is a 0/1 mask of S."""
    lib = lib or _load()
    eu, ev = _edges(g)
    member = np.ascontiguousarray(member, dtype=np.uint8)
    query = np.ascontiguousarray(query, dtype=np.int32)
    out = np.zeros(query.shape[0], np.int64)
    rc = lib.oracle_support_in(g.n_u, g.n_v, g.m, _ptr(eu), _ptr(ev), side, _ptr(member),
                               _ptr(query), query.shape[0], _ptr(out))
    if rc != 0:
        raise ValueError("oracle_support_in: invalid argument")
    return out


def support_levels(g, side: int, theta: np.ndarray, query: np.ndarray, lib=None) -> np.ndarray:
    """int64[len(query), 3]: f_x(S) for each x in ``query`` with S = all of
    the side, {w : theta_w >= theta_x} and {w : theta_w > theta_x}."""
    lib = lib or _load()
    eu, ev = _edges(g)
    theta = np.ascontiguousarray(theta, dtype=np.int64)
    if theta.shape != ((g.n_u if side == 0 else g.n_v),):
        raise ValueError("support_levels: theta must hold one value per vertex of the side")
    query = np.ascontiguousarray(query, dtype=np.int32)
    out = np.zeros((query.shape[0], 3), np.int64)
    rc = lib.oracle_support_levels(g.n_u, g.n_v, g.m, _ptr(eu), _ptr(ev), side, _ptr(theta),
                                   _ptr(query), query.shape[0], _ptr(out))
    if rc != 0:
        raise ValueError("oracle_support_levels: invalid argument")
    return out


def canonical_edges(g, lib=None):
    """(cu int32[m'], cv int32[m']): duplicates merged, sorted by (u, v)."""
    lib = lib or _load()
    eu, ev = _edges(g)
    cu = np.zeros(max(g.m, 1), np.int32)
    cv = np.zeros(max(g.m, 1), np.int32)
    mu = np.zeros(1, np.int64)
    if lib.oracle_canonical_edges(g.n_u, g.n_v, g.m, _ptr(eu), _ptr(ev), _ptr(cu), _ptr(cv), _ptr(mu)) != 0:
        raise ValueError("oracle_canonical_edges: invalid graph")
    k = int(mu[0])
    return cu[:k].copy(), cv[:k].copy()


def edge_count(g, lib=None) -> np.ndarray:
    """Butterflies containing each canonical edge: int64[m']."""
    lib = lib or _load()
    eu, ev = _edges(g)
    k = canonical_edges(g, lib)[0].shape[0]
    out = np.zeros(max(k, 1), np.int64)
    if lib.oracle_edge_count(g.n_u, g.n_v, g.m, _ptr(eu), _ptr(ev), _ptr(out)) != 0:
        raise ValueError("oracle_edge_count: invalid graph")
    return out[:k]


def wing(g, lib=None):
    """Returns (psi int64[m'], peel order int64[m'], pairs examined)."""
    lib = lib or _load()
    eu, ev = _edges(g)
    k = canonical_edges(g, lib)[0].shape[0]
    psi = np.zeros(max(k, 1), np.int64)
    order = np.zeros(max(k, 1), np.int64)
    w = np.zeros(1, np.int64)
    if lib.oracle_wing(g.n_u, g.n_v, g.m, _ptr(eu), _ptr(ev), _ptr(psi), _ptr(order), _ptr(w)) != 0:
        raise ValueError("oracle_wing: invalid graph")
    return psi[:k], order[:k], int(w[0])


def ktip(g, side: int, theta: np.ndarray, k: int, lib=None) -> np.ndarray:
    """k-tips of one side: int32 label per vertex (smallest id of its k-tip,
    -1 when theta < k)."""
    lib = lib or _load()
    eu, ev = _edges(g)
    n = g.n_u if side == 0 else g.n_v
    theta = np.ascontiguousarray(theta, dtype=np.int64)
    if theta.shape != (n,):
        raise ValueError("ktip: one theta per vertex of the side")
    out = np.zeros(max(n, 1), np.int32)
    if lib.oracle_ktip(g.n_u, g.n_v, g.m, _ptr(eu), _ptr(ev), side, _ptr(theta), int(k), _ptr(out)) != 0:
        raise ValueError("oracle_ktip: invalid argument")
    return out[:n]
