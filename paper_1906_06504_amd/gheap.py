"""Python binding of libgheap.so (ctypes).  Argument marshalling only: every
step of the heap runs in the HIP library; PyTorch supplies device memory and
streams.

The library must have been built (``python -m paper_1906_06504_amd.build``);
importing this module without it raises ImportError -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgheap.so")

GH_OK = 0
GH_EINVAL = -1
GH_ENOMEM = -2
GH_ETIMEDOUT = -3
GH_EDEVICE = -4
GH_ESTATE = -5

OP_INSERT = 0
OP_DELETE_MIN = 1
GH_U32_ID = 0    # 8-byte entries: u32 key above u32 id
GH_I64_ID = 1    # 16-byte entries: biased i64 key word, then u32 id and u32 zero
ENTRY_WORDS = {GH_U32_ID: 1, GH_I64_ID: 2}
SUPPORTED_K = (32, 64, 128, 256, 512, 1024)
ENTRY_MAX = 0xFFFFFFFFFFFFFFFF

# struct gh_op / gh_logrec layouts (include/gheap.h)
OP_DTYPE = np.dtype([("heap", "<u4"), ("kind", "<u4"), ("n", "<u4"), ("seq", "<u4"),
                     ("off", "<u8"), ("arrival_ns", "<u8")])
LOG_DTYPE = np.dtype([("ticket", "<u8"), ("count", "<u4"), ("levels", "<u2"), ("kind", "u1"),
                      ("flags", "u1"), ("pb", "<u2"), ("reserved", "<u2"), ("t_claim", "<u4"),
                      ("t_root", "<u4"), ("t_done", "<u4")])
REQ_DTYPE = np.dtype([("first_ticket", "<u8"), ("count", "<u4"), ("nops", "<u2"), ("kind", "u1"),
                      ("flags", "u1"), ("t_admit", "<u4"), ("t_done", "<u4"), ("t_resp", "<u4"),
                      ("bytes", "<u4")])
KNAP_DTYPE = np.dtype([("best", "<u8"), ("explored", "<u8"), ("created", "<u8"),
                       ("popped", "<u8"), ("gc_dropped", "<u8"), ("alg_bytes", "<u8"),
                       ("ops", "<u4"), ("flags", "<u4"), ("gc_runs", "<u4"), ("reserved", "<u4")])
assert OP_DTYPE.itemsize == 32 and LOG_DTYPE.itemsize == 32 and REQ_DTYPE.itemsize == 32
assert KNAP_DTYPE.itemsize == 64
SSSP_DTYPE = np.dtype([("popped", "<u8"), ("stale", "<u8"), ("pushed", "<u8"), ("heap_ops", "<u8"),
                       ("heap_ticks", "<u8"), ("relax_ticks", "<u8"), ("rounds", "<u8"),
                       ("traced", "<u8"), ("alg_bytes", "<u8")])
SSSPOP_DTYPE = np.dtype([("ticket", "<u8"), ("off", "<u8"), ("count", "<u4"), ("kind", "<u4"),
                         ("reserved", "<u8")])
assert SSSP_DTYPE.itemsize == 72 and SSSPOP_DTYPE.itemsize == 32

REQ_ADMITTED = 1
REQ_DEFERRED = 2
REQ_REJECTED = 0x40

FLAG_FULL = 1
FLAG_HANDOFF = 2
FLAG_TOOK = 4
FLAG_ROOT = 8
FLAG_REFILL = 16
FLAG_STOPPED = 0x20
FLAG_REJECTED = 0x40
FLAG_ABORTED = 0x80

EXPORTS = ("heap_arena_bytes", "heap_supported_shape", "heap_create", "heap_create_many",
           "heap_insert", "heap_delete_min", "heap_submit", "heap_submit_graph",
           "heap_graph_launch", "heap_graph_destroy", "heap_sync", "heap_size",
           "heap_read_state", "heap_destroy", "heap_strerror", "heap_clock_hz",
           "heap_serve_workspace_bytes", "heap_serve", "heap_knapsack", "heap_sssp",
           "heap_build", "heap_filter_workspace_bytes", "heap_filter",
           "heap_filter_noalloc", "heap_insert_max")


class GHeapError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__("%s failed: %s (%d)" % (what, strerror(code), code))


_lib = None


GH_TUNE_VARIABLE_DELETE = 1
GH_TUNE_MULTI_INSERT = 2
GH_TUNE_BOTTOM_UP = 4
GH_TUNE_SHARED_ROOT = 8


class _Tuning(ctypes.Structure):
    _fields_ = [("workgroups", ctypes.c_uint32), ("threads", ctypes.c_uint32),
                ("flags", ctypes.c_uint32)]


class SsspTrace(ctypes.Structure):
    """struct gh_sssptrace (device pointers and capacities)."""
    _fields_ = [("d_ops", ctypes.c_void_p), ("op_cap", ctypes.c_uint64),
                ("d_keys", ctypes.c_void_p), ("key_cap", ctypes.c_uint64)]


def load_library(path: str = LIB_PATH):
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libgheap.so is not built at %s; run "
                          "`python -m paper_1906_06504_amd.build`" % path)
    lib = ctypes.CDLL(path)
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    sig = {
        "heap_arena_bytes": (u64, [u32, i32, u32, vp, u64]),
        "heap_supported_shape": (i32, [u32, u32]),
        "heap_create": (i32, [ctypes.POINTER(vp), u32, u64, i32, vp, u64, vp]),
        "heap_create_many": (i32, [ctypes.POINTER(vp), u32, i32, u32, vp, vp, u64, vp]),
        "heap_insert": (i32, [vp, vp, u64]),
        "heap_delete_min": (i32, [vp, vp, u32, vp]),
        "heap_submit": (i32, [vp, vp, u32, vp, vp, vp, vp, ctypes.POINTER(_Tuning)]),
        "heap_submit_graph": (i32, [vp, vp, u32, vp, vp, vp, vp, ctypes.POINTER(_Tuning),
                                    ctypes.POINTER(vp)]),
        "heap_graph_launch": (i32, [vp, vp]),
        "heap_graph_destroy": (i32, [vp]),
        "heap_sync": (i32, [vp]),
        "heap_size": (i32, [vp, u32, ctypes.POINTER(u64)]),
        "heap_read_state": (i32, [vp, u32, vp, vp, vp]),
        "heap_destroy": (i32, [vp]),
        "heap_strerror": (ctypes.c_char_p, [i32]),
        "heap_clock_hz": (u64, []),
        "heap_serve_workspace_bytes": (u64, [u32, u32, u64]),
        "heap_serve": (i32, [vp, vp, u32, vp, vp, vp, vp, u64, u64, ctypes.POINTER(_Tuning)]),
        "heap_knapsack": (i32, [vp, u32, vp, vp, vp, vp, vp, vp, u64, vp, vp, u32,
                                ctypes.POINTER(_Tuning)]),
        "heap_sssp": (i32, [vp, u32, vp, vp, vp, u32, vp, vp, u64, vp,
                            ctypes.POINTER(_Tuning), ctypes.POINTER(SsspTrace)]),
        "heap_build": (i32, [vp, u32, vp, u64]),
        "heap_filter_workspace_bytes": (u64, [vp, u32]),
        "heap_filter": (i32, [vp, u32, u64, vp, u64, vp]),
        "heap_filter_noalloc": (i32, [vp, u32, u64, vp]),
        "heap_insert_max": (u32, [u32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _tune_flags(var_delete: bool, multi_insert: bool, bottom_up: bool = False,
                shared_root: bool = False) -> int:
    return ((GH_TUNE_VARIABLE_DELETE if var_delete else 0) |
            (GH_TUNE_MULTI_INSERT if multi_insert else 0) |
            (GH_TUNE_BOTTOM_UP if bottom_up else 0) |
            (GH_TUNE_SHARED_ROOT if shared_root else 0))


def insert_max(k: int) -> int:
    """Largest insert one operation may hold (heap_insert_max)."""
    return int(load_library().heap_insert_max(k))


def strerror(code: int) -> str:
    return load_library().heap_strerror(code).decode()


def _check(rc: int, what: str):
    if rc != GH_OK:
        raise GHeapError(rc, what)


_U64 = tuple(d for d in (torch.int64, getattr(torch, "uint64", None)) if d is not None)


def _ptr(t, dtypes=None, min_bytes: int = 0, what: str = "tensor") -> int | None:
    """Device address of a contiguous tensor for the C ABI.  The library
    reads and writes device memory by the counts it is given, so the dtype
    (entries are 8 bytes) and the size are checked here, before any launch."""
    if t is None:
        return None
    if dtypes is not None and t.dtype not in dtypes:
        raise TypeError("%s: dtype %s, expected one of %s" % (what, t.dtype, dtypes))
    nbytes = t.numel() * t.element_size()
    if nbytes < min_bytes:
        raise ValueError("%s: %d bytes, at least %d needed" % (what, nbytes, min_bytes))
    if not t.is_cuda:
        raise ValueError("%s: device tensor expected" % what)
    if not t.is_contiguous():
        raise ValueError("%s: contiguous tensor expected" % what)
    return t.data_ptr()


def to_device_u64(a: np.ndarray, device="cuda") -> torch.Tensor:
    """uint64 numpy array -> int64 device tensor holding the same bits (a
    2-D array of 16-byte entries [n, 2] is flattened, entry by entry)."""
    a = np.ascontiguousarray(a, dtype=np.uint64).reshape(-1)
    return torch.from_numpy(a.view(np.int64)).to(device)


def to_host_u64(t: torch.Tensor, ewords: int = 1) -> np.ndarray:
    """Device entries -> uint64 numpy array ([n, 2] for 16-byte entries)."""
    a = t.cpu().numpy().view(np.uint64).reshape(-1)
    return a.reshape(-1, 2) if ewords == 2 else a


def pack_i64(keys, ids) -> np.ndarray:
    """16-byte entries [n, 2] uint64 from signed 64-bit keys and 32-bit ids:
    the key word is the key XOR 2^63 (so it orders as unsigned), the id word
    the id with 32 zero bits above it."""
    k = np.asarray(keys, dtype=np.int64).view(np.uint64) ^ np.uint64(1 << 63)
    i = np.asarray(ids, dtype=np.uint64) & np.uint64(0xFFFFFFFF)
    return np.ascontiguousarray(np.stack([k, i], axis=1))


def unpack_i64(entries):
    """(keys int64, ids uint32) of [n, 2] 16-byte entries."""
    e = np.asarray(entries, dtype=np.uint64).reshape(-1, 2)
    return (e[:, 0] ^ np.uint64(1 << 63)).view(np.int64), (e[:, 1] & np.uint64(0xFFFFFFFF)).astype(np.uint32)


def arena_bytes(k: int, max_keys, keytype: int = GH_U32_ID) -> int:
    lib = load_library()
    mk = np.ascontiguousarray(np.atleast_1d(np.asarray(max_keys, dtype=np.uint64)))
    return int(lib.heap_arena_bytes(k, keytype, mk.size, mk.ctypes.data, 0))


def supported_shape(k: int, threads: int) -> bool:
    return bool(load_library().heap_supported_shape(k, threads))


def clock_hz() -> int:
    return int(load_library().heap_clock_hz())


class HeapSet:
    """One or more device heaps sharing node capacity k, an arena and a stream."""

    def __init__(self, k: int, max_keys, device: str | torch.device = "cuda",
                 stream: torch.cuda.Stream | None = None, keytype: int = GH_U32_ID):
        self.lib = load_library()
        self.k = int(k)
        if keytype not in ENTRY_WORDS:
            raise GHeapError(GH_EINVAL, "keytype")
        self.keytype = int(keytype)
        self.ewords = ENTRY_WORDS[self.keytype]   # 8-byte words per entry
        self.ebytes = 8 * self.ewords
        mk = np.ascontiguousarray(np.atleast_1d(np.asarray(max_keys, dtype=np.uint64)))
        self.nheaps = int(mk.size)
        self.max_keys = mk
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = int(self.lib.heap_arena_bytes(self.k, self.keytype, self.nheaps, mk.ctypes.data, 0))
        if nbytes == 0:
            raise GHeapError(GH_EINVAL, "heap_arena_bytes")
        # 256-byte alignment: torch's caching allocator returns 512-aligned blocks
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        rc = self.lib.heap_create_many(ctypes.byref(h), self.k, self.keytype, self.nheaps,
                                       mk.ctypes.data,
                                       self.arena.data_ptr(), nbytes,
                                       ctypes.c_void_p(self.stream.cuda_stream))
        _check(rc, "heap_create_many")
        self.h = h
        self._graphs = []

    # -- single-heap calls (heap 0) -------------------------------------
    def insert(self, keys: torch.Tensor) -> None:
        """Insert a contiguous int64/uint64 device tensor of entries (one
        word an entry, or two for 16-byte entries) into heap 0."""
        _check(self.lib.heap_insert(self.h, _ptr(keys, _U64, what="keys"),
                                    keys.numel() // self.ewords), "heap_insert")

    def delete_min(self, out: torch.Tensor | None = None, count: torch.Tensor | None = None,
                   c: int | None = None):
        """deleteMin of c entries (default k) on heap 0; returns (out int64
        tensor with room for c, count int32 tensor)."""
        c = self.k if c is None else int(c)
        if out is None:
            out = torch.empty(max(c, 1) * self.ewords, dtype=torch.int64, device=self.device)
        if count is None:
            count = torch.zeros(1, dtype=torch.int32, device=self.device)
        _check(self.lib.heap_delete_min(self.h, _ptr(out, _U64, self.ebytes * c, "out"), c,
                                        _ptr(count, (torch.int32,), 4, "count")),
               "heap_delete_min")
        return out, count

    # -- submissions -------------------------------------------------------
    def submit(self, ops: torch.Tensor, nops: int, d_in: torch.Tensor | None,
               d_out: torch.Tensor | None, counts: torch.Tensor | None = None,
               log: torch.Tensor | None = None, workgroups: int = 0, threads: int = 0,
               var_delete: bool = False, multi_insert: bool = False, bottom_up: bool = False,
               shared_root: bool = False):
        """Run the op records on the set's stream.  var_delete: the records
        may hold deleteMins of fewer than k entries (n in 1..k-1);
        multi_insert: inserts of more than k entries (up to insert_max(k));
        bottom_up: every record is an insert of up to k entries, run
        bottom-up (GH_TUNE_BOTTOM_UP); shared_root: with one workgroup, the
        per-operation root protocol instead of the lock-free one-workgroup
        loop (GH_TUNE_SHARED_ROOT)."""
        t = _Tuning(workgroups, threads,
                    _tune_flags(var_delete, multi_insert, bottom_up, shared_root))
        rc = self.lib.heap_submit(self.h, *self._op_ptrs(ops, nops, d_in, d_out, counts, log),
                                  ctypes.byref(t))
        _check(rc, "heap_submit")

    def submit_graph(self, ops, nops, d_in, d_out, counts=None, log=None, workgroups=0,
                     threads=0, var_delete: bool = False, multi_insert: bool = False) -> int:
        t = _Tuning(workgroups, threads, _tune_flags(var_delete, multi_insert))
        g = ctypes.c_void_p()
        rc = self.lib.heap_submit_graph(self.h, *self._op_ptrs(ops, nops, d_in, d_out, counts,
                                                               log),
                                        ctypes.byref(t), ctypes.byref(g))
        _check(rc, "heap_submit_graph")
        self._graphs.append(g.value)
        return g.value

    @staticmethod
    def _op_ptrs(ops, nops, d_in, d_out, counts, log):
        """Arguments of heap_submit after the handle: the records, their count
        and the buffers.  Entry buffers are addressed by the records' offsets,
        so only their dtype is checked; per-operation arrays by nops."""
        nops = int(nops)
        return (_ptr(ops, None, nops * OP_DTYPE.itemsize, "ops"), nops,
                _ptr(d_in, _U64, 0, "d_in"), _ptr(d_out, _U64, 0, "d_out"),
                _ptr(counts, (torch.int32,), 4 * nops, "counts"),
                _ptr(log, None, nops * LOG_DTYPE.itemsize, "log"))

    def graph_launch(self, g: int) -> None:
        _check(self.lib.heap_graph_launch(self.h, ctypes.c_void_p(g)), "heap_graph_launch")

    def serve(self, reqs: torch.Tensor, nreq: int, d_in: torch.Tensor | None,
              d_out: torch.Tensor | None, recs: torch.Tensor, max_ops: int,
              work: torch.Tensor | None = None, workgroups: int = 0, threads: int = 0,
              multi_insert: bool = False):
        """Run a request stream through the device-resident serving loop
        (multi_insert: inserts of up to insert_max(k) entries take the root
        once, GH_TUNE_MULTI_INSERT).  Returns the workspace tensor (reusable
        for the next call)."""
        need = int(self.lib.heap_serve_workspace_bytes(self.nheaps, nreq, max_ops))
        if work is None or work.numel() < need:
            work = torch.empty(need, dtype=torch.uint8, device=self.device)
        t = _Tuning(workgroups, threads, GH_TUNE_MULTI_INSERT if multi_insert else 0)
        rc = self.lib.heap_serve(self.h, _ptr(reqs, None, nreq * OP_DTYPE.itemsize, "reqs"), nreq,
                                 _ptr(d_in, _U64, 0, "d_in"), _ptr(d_out, _U64, 0, "d_out"),
                                 _ptr(recs, None, nreq * REQ_DTYPE.itemsize, "recs"),
                                 _ptr(work, (torch.uint8,), need, "work"), work.numel(), max_ops,
                                 ctypes.byref(t))
        _check(rc, "heap_serve")
        return work

    def build(self, i: int, sorted_keys: torch.Tensor):
        """Bulk-build empty heap i from an ascending int64 tensor of entries."""
        _check(self.lib.heap_build(self.h, i, _ptr(sorted_keys, _U64, what="sorted_keys"),
                                   sorted_keys.numel() // self.ewords), "heap_build")

    def filter(self, i: int, bound: int, work: torch.Tensor | None = None):
        """Remove every entry >= bound from heap i (stream-ordered).  Returns
        (kept: int64 device tensor of one element, workspace for reuse)."""
        need = int(self.lib.heap_filter_workspace_bytes(self.h, i))
        if need == 0:
            raise GHeapError(GH_EINVAL, "heap_filter_workspace_bytes")
        if work is None or work.numel() < need:
            work = torch.empty(need, dtype=torch.uint8, device=self.device)
        kept = torch.zeros(1, dtype=torch.int64, device=self.device)
        _check(self.lib.heap_filter(self.h, i, int(bound), _ptr(work, (torch.uint8,), need, "work"),
                                    work.numel(),
                                    _ptr(kept)), "heap_filter")
        return kept, work

    def filter_noalloc(self, i: int, bound: int, kept: torch.Tensor | None = None):
        """heap_filter without a workspace: the library's own device array
        is the workspace.  Returns kept (int64 device tensor of one element)."""
        if kept is None:
            kept = torch.zeros(1, dtype=torch.int64, device=self.device)
        _check(self.lib.heap_filter_noalloc(self.h, i, int(bound), _ptr(kept, _U64, 8, "kept")),
               "heap_filter_noalloc", "heap_insert_max")
        return kept

    def sync(self) -> int:
        return int(self.lib.heap_sync(self.h))

    def size(self, i: int = 0) -> int:
        v = ctypes.c_uint64()
        _check(self.lib.heap_size(self.h, i, ctypes.byref(v)), "heap_size")
        return int(v.value)

    def read_state(self, i: int = 0):
        """(m, s, served, max_nodes, nodes[max_nodes, k] uint64, pb[s] uint64);
        16-byte entries: nodes[max_nodes, k, 2], pb[s, 2]."""
        meta = np.zeros(4, dtype=np.uint64)
        _check(self.lib.heap_read_state(self.h, i, meta.ctypes.data, None, None),
               "heap_read_state")
        w = self.ewords
        nodes = np.empty(int(meta[3]) * self.k * w, dtype=np.uint64)
        pb = np.empty(max(int(meta[1]), 1) * w, dtype=np.uint64)
        _check(self.lib.heap_read_state(self.h, i, meta.ctypes.data, nodes.ctypes.data,
                                        pb.ctypes.data), "heap_read_state")
        shape = (int(meta[3]), self.k) + ((2,) if w == 2 else ())
        pb = pb.reshape(-1, 2) if w == 2 else pb
        return (int(meta[0]), int(meta[1]), int(meta[2]), int(meta[3]),
                nodes.reshape(shape), pb[: int(meta[1])].copy())

    def close(self) -> int:
        rc = GH_OK
        if getattr(self, "h", None):
            for g in self._graphs:
                self.lib.heap_graph_destroy(ctypes.c_void_p(g))
            self._graphs = []
            rc = int(self.lib.heap_destroy(self.h))
            self.h = None
        return rc

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Heap(HeapSet):
    """A single device heap (heap_create)."""

    def __init__(self, k: int, max_keys: int, device="cuda", stream=None, keytype=GH_U32_ID):
        super().__init__(k, [max_keys], device=device, stream=stream, keytype=keytype)


def ops_to_device(oplist, device="cuda"):
    """Pack a workloads.OpList into gh_op records on the device.
    Returns (ops tensor, nops, keys tensor, out tensor, counts tensor)."""
    n = len(oplist)
    rec = np.zeros(n, dtype=OP_DTYPE)
    rec["heap"] = oplist.heap_ids()
    rec["kind"] = oplist.kind
    rec["n"] = oplist.n
    rec["seq"] = oplist.seq()
    rec["off"] = oplist.off
    if oplist.arrival is not None:
        rec["arrival_ns"] = oplist.arrival
    ops = torch.from_numpy(rec.view(np.uint8).copy()).to(device)
    w = entry_words(oplist)
    keys = to_device_u64(oplist.keys if oplist.keys.size else np.zeros(w, np.uint64), device)
    out = torch.full((max(oplist.out_entries, 1) * w,), -1, dtype=torch.int64, device=device)
    counts = torch.zeros(max(n, 1), dtype=torch.int32, device=device)
    return ops, n, keys, out, counts


def entry_words(oplist) -> int:
    """8-byte words per entry of an op list: 2 when its keys are [n, 2]."""
    return 2 if oplist.keys.ndim == 2 else 1


def new_log(nops: int, device="cuda") -> torch.Tensor:
    return torch.zeros(max(nops, 1) * LOG_DTYPE.itemsize, dtype=torch.uint8, device=device)


def log_to_host(log: torch.Tensor, nops: int) -> np.ndarray:
    return log.cpu().numpy().view(LOG_DTYPE)[:nops].copy()


def requests_to_device(oplist, device="cuda"):
    """Pack a request stream (workloads.OpList with heap ids and arrivals)
    into gh_op records on the device.  Returns (reqs, nreq, keys, out, recs,
    max_ops) where max_ops bounds the operations the stream can expand to."""
    n = len(oplist)
    rec = np.zeros(n, dtype=OP_DTYPE)
    rec["heap"] = oplist.heap_ids()
    rec["kind"] = oplist.kind
    rec["n"] = oplist.n
    rec["off"] = oplist.off
    if oplist.arrival is not None:
        rec["arrival_ns"] = oplist.arrival
    k = int(oplist.meta.get("k", 1))
    ins = oplist.kind == OP_INSERT
    # insert requests become operations of up to heap_insert_max(k) entries,
    # or of k entries with split inserts: bound by the latter
    max_ops = int(np.sum(-(-oplist.n[ins].astype(np.int64) // k))) + int((~ins).sum())
    reqs = torch.from_numpy(rec.view(np.uint8).copy()).to(device)
    w = entry_words(oplist)
    keys = to_device_u64(oplist.keys if oplist.keys.size else np.zeros(w, np.uint64), device)
    out = torch.full((max(oplist.out_entries, 1) * w,), -1, dtype=torch.int64, device=device)
    recs = torch.zeros(max(n, 1) * REQ_DTYPE.itemsize, dtype=torch.uint8, device=device)
    return reqs, n, keys, out, recs, max(max_ops, 1)


def recs_to_host(recs: torch.Tensor, nreq: int) -> np.ndarray:
    return recs.cpu().numpy().view(REQ_DTYPE)[:nreq].copy()
