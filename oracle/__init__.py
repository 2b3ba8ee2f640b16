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
MAXE = np.uint64(0xFFFFFFFFFFFFFFFF)


def build(force: bool = True) -> str:
    """Compile the oracle C sources into liboracle.so (gcc, -O2): the heap
    oracle twice, for 8-byte entries (gho_*) and for 16-byte entries
    (-DGHO_WIDE, ghow_*), and the application oracles."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    srcs = [os.path.join(_HERE, s) for s in _SOURCES if os.path.exists(os.path.join(_HERE, s))]
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    flags = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC"]
    objs = []
    for i, src in enumerate(srcs + [os.path.join(_HERE, "gheap_oracle.c")]):
        obj = tmp + ".%d.o" % i
        wide = ["-DGHO_WIDE"] if i == len(srcs) else []
        subprocess.check_call(flags + wide + ["-c", src, "-o", obj])
        objs.append(obj)
    try:
        subprocess.check_call(["gcc", "-shared", "-o", tmp] + objs)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
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
    _declare_heap(lib, "gho_")
    if hasattr(lib, "ghow_new"):
        _declare_heap(lib, "ghow_")
        lib.ghow_filter_key.restype = ctypes.c_uint64
        lib.ghow_filter_key.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
    if hasattr(lib, "gho_dijkstra"):
        lib.gho_dijkstra.restype = ctypes.c_int
        lib.gho_dijkstra.argtypes = [ctypes.c_uint32, U64P, U32P, U32P, ctypes.c_uint32, U32P]
    if hasattr(lib, "gho_knapsack_dp"):
        lib.gho_knapsack_dp.restype = ctypes.c_uint64
        lib.gho_knapsack_dp.argtypes = [ctypes.c_uint32, U32P, U32P, ctypes.c_uint64]
    return lib


def _declare_heap(lib, pre):
    """Signatures of one entry width's heap functions (entry pointers are
    passed as void pointers: 8 or 16 bytes an entry)."""
    EP = ctypes.c_void_p
    f = lambda name: getattr(lib, pre + name)  # noqa: E731
    f("new").restype = ctypes.c_void_p
    f("new").argtypes = [ctypes.c_uint32]
    f("free").restype = None
    f("free").argtypes = [ctypes.c_void_p]
    for name in ("size", "nodes", "pb_size", "node_slots"):
        f(name).restype = ctypes.c_uint64
        f(name).argtypes = [ctypes.c_void_p]
    f("idx").restype = ctypes.c_uint64
    f("idx").argtypes = [ctypes.c_uint64]
    f("insert").restype = ctypes.c_int
    f("insert").argtypes = [ctypes.c_void_p, EP, ctypes.c_uint64]
    if hasattr(lib, pre + "insert_bu"):
        f("insert_bu").restype = ctypes.c_int
        f("insert_bu").argtypes = [ctypes.c_void_p, EP, ctypes.c_uint64]
    f("delete_min").restype = ctypes.c_uint64
    f("delete_min").argtypes = [ctypes.c_void_p, EP]
    f("delete_min_n").restype = ctypes.c_uint64
    f("delete_min_n").argtypes = [ctypes.c_void_p, EP, ctypes.c_uint64]
    f("build").restype = ctypes.c_int
    f("build").argtypes = [ctypes.c_void_p, EP, ctypes.c_uint64]
    f("check").restype = ctypes.c_int
    f("check").argtypes = [ctypes.c_void_p]
    f("export").restype = None
    f("export").argtypes = [ctypes.c_void_p, EP, EP]
    f("counters").restype = None
    f("counters").argtypes = [ctypes.c_void_p, U64P]
    f("replay").restype = ctypes.c_int64
    f("replay").argtypes = [ctypes.c_void_p, ctypes.c_uint64, U8P, U32P, U64P, EP, EP, U32P,
                            ctypes.c_int]
    f("merge_and_sort").restype = None
    f("merge_and_sort").argtypes = [ctypes.c_void_p, EP, ctypes.c_uint64, EP, ctypes.c_uint64,
                                    EP, EP]
    if pre == "gho_":
        f("filter").restype = ctypes.c_uint64
        f("filter").argtypes = [ctypes.c_void_p, ctypes.c_uint64]


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


def _vp(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def wide_to_c(a) -> np.ndarray:
    """16-byte entries from the device layout ([n, 2] uint64: key word, id
    word) to the oracle's (an unsigned 128-bit integer, low half first in
    memory: id word, key word)."""
    a = np.asarray(a, dtype=np.uint64).reshape(-1, 2)
    return np.ascontiguousarray(a[:, ::-1])


def wide_from_c(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64).reshape(-1, 2)[:, ::-1])


class OracleHeap:
    """Sequential generalized heap with node capacity k (any k >= 1).

    wide=False: 8-byte entries, 1-D uint64 arrays.  wide=True: 16-byte
    entries as [n, 2] uint64 arrays in the device layout (biased key word,
    id word), ordered by key word, then id word."""

    def __init__(self, k: int, lib=None, wide: bool = False):
        self.lib = lib if lib is not None else load()
        self.k = int(k)
        self.wide = bool(wide)
        self.pre = "ghow_" if self.wide else "gho_"
        self.h = self._f("new")(self.k)
        if not self.h:
            raise MemoryError("gho_new failed")

    def _f(self, name):
        return getattr(self.lib, self.pre + name)

    def _in(self, keys) -> np.ndarray:
        """Caller entries -> the oracle's C layout (contiguous)."""
        if self.wide:
            return wide_to_c(keys)
        return np.ascontiguousarray(np.asarray(keys, dtype=np.uint64).reshape(-1))

    def _out(self, a: np.ndarray) -> np.ndarray:
        return wide_from_c(a) if self.wide else a

    def _empty(self, n: int) -> np.ndarray:
        return np.empty((max(n, 1), 2) if self.wide else max(n, 1), dtype=np.uint64)

    def close(self):
        if self.h:
            self._f("free")(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def insert(self, keys, bottom_up: bool = False) -> None:
        """Insert keys (chunks of k); bottom_up: each full batch climbs from
        its target (the bottom-up INS) instead of descending from the root."""
        a = self._in(keys)
        n = a.shape[0]
        if n and np.any(np.all(a.reshape(n, -1) == MAXE, axis=1)):
            raise ValueError("the all-ones entry is reserved")
        if self._f("insert_bu" if bottom_up else "insert")(self.h, _vp(a) if n else None, n) != 0:
            raise MemoryError("gho_insert failed")

    def delete_min(self, c: int | None = None) -> np.ndarray:
        """Remove and return the min(c, size) smallest entries (c = k when
        None; 1 <= c <= k)."""
        out = self._empty(self.k)
        if c is None:
            got = self._f("delete_min")(self.h, _vp(out))
        else:
            got = self._f("delete_min_n")(self.h, _vp(out), int(c))
            if got == 0xFFFFFFFFFFFFFFFF:
                raise ValueError("deleteMin count must be in [1, k]")
        return self._out(out[:got]).copy()

    def build(self, sorted_keys) -> None:
        """Bulk build of an empty heap from ascending entries (Sec. 3.1)."""
        a = self._in(sorted_keys)
        rc = self._f("build")(self.h, _vp(a) if a.shape[0] else None, a.shape[0])
        if rc == -2:
            raise ValueError("entries must be ascending and not the reserved value")
        if rc != 0:
            raise RuntimeError("gho_build failed (heap not empty or no memory)")

    def filter(self, bound: int) -> int:
        """Remove every entry >= bound (16-byte entries: every entry whose
        key word is >= bound); returns the number kept."""
        if self.wide:
            kept = self.lib.ghow_filter_key(self.h, int(bound))
        else:
            kept = self.lib.gho_filter(self.h, int(bound))
        if kept == 0xFFFFFFFFFFFFFFFF:
            raise MemoryError("gho_filter failed")
        return int(kept)

    def check(self) -> int:
        return int(self._f("check")(self.h))

    @property
    def size(self) -> int:
        return int(self._f("size")(self.h))

    @property
    def m(self) -> int:
        return int(self._f("nodes")(self.h))

    @property
    def s(self) -> int:
        return int(self._f("pb_size")(self.h))

    def export(self):
        """Return (nodes[slots, k], pb[s]) copies of the internal state
        (16-byte entries: nodes[slots, k, 2], pb[s, 2] in the device layout)."""
        slots = int(self._f("node_slots")(self.h))
        nodes = self._empty(slots * self.k)
        pb = self._empty(self.s)
        self._f("export")(self.h, _vp(nodes), _vp(pb))
        if self.wide:
            return (self._out(nodes).reshape(slots, self.k, 2), self._out(pb)[: self.s].copy())
        return nodes.reshape(slots, self.k), pb[: self.s].copy()

    def counters(self) -> dict:
        c = np.zeros(7, dtype=np.uint64)
        self._f("counters")(self.h, _p64(c))
        return dict(ins_ops=int(c[0]), ins_full=int(c[1]), ins_path_nodes=int(c[2]),
                    del_ops=int(c[3]), del_levels=int(c[4]), del_refill=int(c[5]),
                    traffic_entries=int(c[6]))

    def replay(self, types, n, off, in_keys, out_capacity: int, check: bool = False):
        """Apply ops in order (type 0 = INS n[i] keys from in_keys[off[i]:],
        type 1 = DEL of n[i] entries (0 = k) writing to out[off[i]:]).
        Returns (out_keys, counts)."""
        types = np.ascontiguousarray(types, dtype=np.uint8)
        n = np.ascontiguousarray(n, dtype=np.uint32)
        off = np.ascontiguousarray(off, dtype=np.uint64)
        keys = self._in(in_keys)
        if keys.shape[0] == 0:
            keys = self._empty(1)
        out = self._empty(out_capacity)
        out.fill(np.uint64(0xFFFFFFFFFFFFFFFF))
        counts = np.zeros(types.size, dtype=np.uint32)
        rc = self._f("replay")(self.h, types.size, types.ctypes.data_as(U8P), _p32(n), _p64(off),
                               _vp(keys), _vp(out), _p32(counts), 1 if check else 0)
        if rc != 0:
            raise RuntimeError("oracle replay failed at op %d" % (-rc - 1))
        return self._out(out), counts


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
    h = OracleHeap(max(a.size, b.size, 1))
    hi = np.empty(max(a.size, 1), dtype=np.uint64)
    lo = np.empty(max(b.size, 1), dtype=np.uint64)
    aa = a if a.size else np.zeros(1, dtype=np.uint64)
    bb = b if b.size else np.zeros(1, dtype=np.uint64)
    lib.gho_merge_and_sort(h.h, _vp(aa), a.size, _vp(bb), b.size, _vp(hi), _vp(lo))
    return hi[: a.size].copy(), lo[: b.size].copy()
