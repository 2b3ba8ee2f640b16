"""Plain CPU oracle for the generalized concurrent heap.

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` are the only callers.  The HIP library and its
Python binding never import this package, and this package never imports
them.

The C sources in this directory are compiled into ``liboracle.so`` with gcc
(``build()``); this module wraps them with ctypes and numpy.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["gheap_oracle.c", "apps_oracle.c"]
_lock = threading.Lock()
_lib = None

U64P = ctypes.POINTER(ctypes.c_uint64)
U32P = ctypes.POINTER(ctypes.c_uint32)
U8P = ctypes.POINTER(ctypes.c_uint8)


def build(force: bool = True) -> str:
    """Compile the oracle C sources into liboracle.so (gcc, -O2)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    srcs = [os.path.join(_HERE, s) for s in _SOURCES if os.path.exists(os.path.join(_HERE, s))]
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", "-o", tmp] + srcs
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def build_variant(defines: list[str], out_name: str) -> str:
    """Compile a variant of the oracle with extra -D flags (used by the tests
    that plant a mistake in the oracle and check that the pins catch it)."""
    out = os.path.join(_HERE, out_name)
    srcs = [os.path.join(_HERE, s) for s in _SOURCES if os.path.exists(os.path.join(_HERE, s))]
    cmd = ["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", out] + ["-D" + d for d in defines] + srcs
    subprocess.check_call(cmd)
    return out


def _declare(lib):
    lib.gho_new.restype = ctypes.c_void_p
    lib.gho_new.argtypes = [ctypes.c_uint32]
    lib.gho_free.restype = None
    lib.gho_free.argtypes = [ctypes.c_void_p]
    for name in ("gho_size", "gho_nodes", "gho_pb_size", "gho_node_slots"):
        f = getattr(lib, name)
        f.restype = ctypes.c_uint64
        f.argtypes = [ctypes.c_void_p]
    lib.gho_idx.restype = ctypes.c_uint64
    lib.gho_idx.argtypes = [ctypes.c_uint64]
    lib.gho_insert.restype = ctypes.c_int
    lib.gho_insert.argtypes = [ctypes.c_void_p, U64P, ctypes.c_uint64]
    lib.gho_delete_min.restype = ctypes.c_uint64
    lib.gho_delete_min.argtypes = [ctypes.c_void_p, U64P]
    lib.gho_delete_min_n.restype = ctypes.c_uint64
    lib.gho_delete_min_n.argtypes = [ctypes.c_void_p, U64P, ctypes.c_uint64]
    lib.gho_build.restype = ctypes.c_int
    lib.gho_build.argtypes = [ctypes.c_void_p, U64P, ctypes.c_uint64]
    lib.gho_filter.restype = ctypes.c_uint64
    lib.gho_filter.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
    lib.gho_check.restype = ctypes.c_int
    lib.gho_check.argtypes = [ctypes.c_void_p]
    lib.gho_export.restype = None
    lib.gho_export.argtypes = [ctypes.c_void_p, U64P, U64P]
    lib.gho_counters.restype = None
    lib.gho_counters.argtypes = [ctypes.c_void_p, U64P]
    lib.gho_replay.restype = ctypes.c_int64
    lib.gho_replay.argtypes = [ctypes.c_void_p, ctypes.c_uint64, U8P, U32P, U64P,
                               U64P, U64P, U32P, ctypes.c_int]
    if hasattr(lib, "gho_dijkstra"):
        lib.gho_dijkstra.restype = ctypes.c_int
        lib.gho_dijkstra.argtypes = [ctypes.c_uint32, U64P, U32P, U32P, ctypes.c_uint32, U32P]
    if hasattr(lib, "gho_knapsack_dp"):
        lib.gho_knapsack_dp.restype = ctypes.c_uint64
        lib.gho_knapsack_dp.argtypes = [ctypes.c_uint32, U32P, U32P, ctypes.c_uint64]
    return lib


def load(path: str | None = None):
    """Load liboracle.so, compiling it first if it is not there."""
    global _lib
    if path is not None:
        return _declare(ctypes.CDLL(path))
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build()
            _lib = _declare(ctypes.CDLL(_LIB_PATH))
    return _lib


def _p64(a: np.ndarray):
    return a.ctypes.data_as(U64P)


def _p32(a: np.ndarray):
    return a.ctypes.data_as(U32P)


def idx(p: int) -> int:
    """Node index of the p-th node added, in bit-reversal order."""
    return int(load().gho_idx(p))


class OracleHeap:
    """Sequential generalized heap with node capacity k (any k >= 1)."""

    def __init__(self, k: int, lib=None):
        self.lib = lib if lib is not None else load()
        self.k = int(k)
        self.h = self.lib.gho_new(self.k)
        if not self.h:
            raise MemoryError("gho_new failed")

    def close(self):
        if self.h:
            self.lib.gho_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def insert(self, keys) -> None:
        a = np.ascontiguousarray(np.asarray(keys, dtype=np.uint64))
        if a.size and np.any(a == np.uint64(0xFFFFFFFFFFFFFFFF)):
            raise ValueError("the all-ones entry is reserved")
        if self.lib.gho_insert(self.h, _p64(a), a.size) != 0:
            raise MemoryError("gho_insert failed")

    def delete_min(self, c: int | None = None) -> np.ndarray:
        """Remove and return the min(c, size) smallest entries (c = k when
        None; 1 <= c <= k)."""
        out = np.empty(self.k, dtype=np.uint64)
        if c is None:
            got = self.lib.gho_delete_min(self.h, _p64(out))
        else:
            got = self.lib.gho_delete_min_n(self.h, _p64(out), int(c))
            if got == 0xFFFFFFFFFFFFFFFF:
                raise ValueError("deleteMin count must be in [1, k]")
        return out[:got].copy()

    def build(self, sorted_keys) -> None:
        """Bulk build of an empty heap from ascending entries (Sec. 3.1)."""
        a = np.ascontiguousarray(np.asarray(sorted_keys, dtype=np.uint64))
        rc = self.lib.gho_build(self.h, _p64(a) if a.size else None, a.size)
        if rc == -2:
            raise ValueError("entries must be ascending and not the reserved value")
        if rc != 0:
            raise RuntimeError("gho_build failed (heap not empty or no memory)")

    def filter(self, bound: int) -> int:
        """Remove every entry >= bound; returns the number kept."""
        kept = self.lib.gho_filter(self.h, int(bound))
        if kept == 0xFFFFFFFFFFFFFFFF:
            raise MemoryError("gho_filter failed")
        return int(kept)

    def check(self) -> int:
        return int(self.lib.gho_check(self.h))

    @property
    def size(self) -> int:
        return int(self.lib.gho_size(self.h))

    @property
    def m(self) -> int:
        return int(self.lib.gho_nodes(self.h))

    @property
    def s(self) -> int:
        return int(self.lib.gho_pb_size(self.h))

    def export(self):
        """Return (nodes[slots, k], pb[s]) copies of the internal state."""
        slots = int(self.lib.gho_node_slots(self.h))
        nodes = np.empty(slots * self.k, dtype=np.uint64)
        pb = np.empty(max(self.s, 1), dtype=np.uint64)
        self.lib.gho_export(self.h, _p64(nodes), _p64(pb))
        return nodes.reshape(slots, self.k), pb[: self.s].copy()

    def counters(self) -> dict:
        c = np.zeros(5, dtype=np.uint64)
        self.lib.gho_counters(self.h, _p64(c))
        return dict(ins_ops=int(c[0]), ins_full=int(c[1]), ins_path_nodes=int(c[2]),
                    del_ops=int(c[3]), del_levels=int(c[4]))

    def replay(self, types, n, off, in_keys, out_capacity: int, check: bool = False):
        """Apply ops in order (type 0 = INS n[i] keys from in_keys[off[i]:],
        type 1 = DEL of n[i] entries (0 = k) writing to out[off[i]:]).
        Returns (out_keys, counts)."""
        types = np.ascontiguousarray(types, dtype=np.uint8)
        n = np.ascontiguousarray(n, dtype=np.uint32)
        off = np.ascontiguousarray(off, dtype=np.uint64)
        in_keys = np.ascontiguousarray(in_keys, dtype=np.uint64)
        if in_keys.size == 0:
            in_keys = np.zeros(1, dtype=np.uint64)
        out = np.full(max(out_capacity, 1), np.uint64(0xFFFFFFFFFFFFFFFF), dtype=np.uint64)
        counts = np.zeros(types.size, dtype=np.uint32)
        rc = self.lib.gho_replay(self.h, types.size, types.ctypes.data_as(U8P), _p32(n),
                                 _p64(off), _p64(in_keys), _p64(out), _p32(counts),
                                 1 if check else 0)
        if rc != 0:
            raise RuntimeError("oracle replay failed at op %d" % (-rc - 1))
        return out, counts


def dijkstra(V: int, rowptr: np.ndarray, col: np.ndarray, w: np.ndarray, src: int) -> np.ndarray:
    """Single-source shortest paths (uint32 distances, UINT32_MAX = unreachable)."""
    lib = load()
    rowptr = np.ascontiguousarray(rowptr, dtype=np.uint64)
    col = np.ascontiguousarray(col, dtype=np.uint32)
    w = np.ascontiguousarray(w, dtype=np.uint32)
    dist = np.empty(V, dtype=np.uint32)
    rc = lib.gho_dijkstra(V, _p64(rowptr), _p32(col), _p32(w), src, _p32(dist))
    if rc != 0:
        raise RuntimeError("dijkstra failed")
    return dist


def knapsack_dp(weights, values, capacity: int) -> int:
    """Optimal 0/1 knapsack value by dynamic programming over capacities."""
    lib = load()
    w = np.ascontiguousarray(weights, dtype=np.uint32)
    v = np.ascontiguousarray(values, dtype=np.uint32)
    return int(lib.gho_knapsack_dp(w.size, _p32(w), _p32(v), capacity))


def merge_and_sort(a, b):
    """MergeAndSort of two sorted runs: (the |a| smallest, the rest)."""
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    lib = load()
    lib.gho_merge_and_sort.restype = None
    lib.gho_merge_and_sort.argtypes = [ctypes.c_void_p, U64P, ctypes.c_uint64, U64P,
                                       ctypes.c_uint64, U64P, U64P]
    h = OracleHeap(max(a.size, b.size, 1))
    hi = np.empty(max(a.size, 1), dtype=np.uint64)
    lo = np.empty(max(b.size, 1), dtype=np.uint64)
    aa = a if a.size else np.zeros(1, dtype=np.uint64)
    bb = b if b.size else np.zeros(1, dtype=np.uint64)
    lib.gho_merge_and_sort(h.h, _p64(aa), a.size, _p64(bb), b.size, _p64(hi), _p64(lo))
    return hi[: a.size].copy(), lo[: b.size].copy()
