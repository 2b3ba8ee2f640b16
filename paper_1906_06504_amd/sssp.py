"""Single-source shortest paths with a device heap as the shared priority
queue (the application of Sec. 5.7.1): host-side preparation and the call
into heap_sssp.  The search itself runs in the HIP library."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import gheap as G


def _dev_u32(a: np.ndarray, device) -> torch.Tensor:
    a = np.ascontiguousarray(a, dtype=np.uint32)
    if a.size == 0:
        a = np.zeros(1, np.uint32)
    return torch.from_numpy(a.view(np.int32)).to(device)


class Graph:
    """A CSR graph resident in device memory."""

    def __init__(self, rowptr: np.ndarray, col: np.ndarray, w: np.ndarray, device="cuda"):
        self.V = int(rowptr.size - 1)
        self.E = int(rowptr[-1])
        if self.V <= 0 or self.V >= (1 << 32) - 1:
            raise ValueError("vertex count out of range")
        if col.size != self.E or w.size != self.E or int(rowptr[0]) != 0:
            raise ValueError("CSR arrays disagree")
        if np.any(np.diff(rowptr.astype(np.int64)) < 0):
            raise ValueError("rowptr must be non-decreasing")
        if self.E and int(np.max(col)) >= self.V:
            raise ValueError("edge target out of range")
        self.max_degree = int(np.max(np.diff(rowptr.astype(np.int64)))) if self.V else 0
        self.rowptr = _dev_u32(rowptr, device)
        self.col = _dev_u32(col, device)
        self.w = _dev_u32(w, device)


class Solver:
    """Heap, push buffers, distances and counters for one graph."""

    def __init__(self, graph: Graph, k: int, workgroups: int = 256, threads: int = 0,
                 device="cuda", stream=None):
        self.g = graph
        self.k = k
        # the push buffer is sized per workgroup; 0 means the library's 256
        self.workgroups = int(workgroups) if workgroups > 0 else 256
        self.threads = threads
        self.hs = G.HeapSet(k, [graph.E + 1], device=device, stream=stream)
        self.push_per_wg = max(1, k * max(1, graph.max_degree))
        self.push = torch.empty(self.workgroups * (self.push_per_wg + k), dtype=torch.int64,
                                device=device)
        self.dist = torch.empty(max(1, graph.V), dtype=torch.int32, device=device)
        self.stats = torch.zeros(G.SSSP_DTYPE.itemsize, dtype=torch.uint8, device=device)

    def launch(self, src: int = 0, trace=None):
        """Enqueue a run on the heap set's stream (no synchronization).
        `trace`: (ops uint8 tensor, keys int64 tensor) to record every heap
        operation, or None."""
        t = G._Tuning(self.workgroups, self.threads)
        tr = None
        if trace is not None:
            ops, keys = trace
            tr = ctypes.byref(G.SsspTrace(ops.data_ptr(), ops.numel() // G.SSSPOP_DTYPE.itemsize,
                                          keys.data_ptr(), keys.numel()))
        rc = self.hs.lib.heap_sssp(self.hs.h, self.g.V, self.g.rowptr.data_ptr(),
                                   self.g.col.data_ptr(), self.g.w.data_ptr(), src,
                                   self.dist.data_ptr(), self.push.data_ptr(), self.push_per_wg,
                                   self.stats.data_ptr(), ctypes.byref(t), tr)
        G._check(rc, "heap_sssp")

    def run(self, src: int = 0, trace=None):
        """Solve; returns (distances as uint32 numpy, counters record)."""
        self.launch(src, trace)
        rc = self.hs.sync()
        if rc != G.GH_OK:
            raise G.GHeapError(rc, "heap_sssp (device)")
        d = self.dist.cpu().numpy().view(np.uint32)[: self.g.V].copy()
        s = self.stats.cpu().numpy().view(G.SSSP_DTYPE)[0].copy()
        return d, s

    def new_trace(self, op_cap: int, key_cap: int):
        """Device buffers for a trace of up to op_cap operations and key_cap
        entries."""
        ops = torch.zeros(op_cap * G.SSSPOP_DTYPE.itemsize, dtype=torch.uint8,
                          device=self.dist.device)
        keys = torch.zeros(key_cap, dtype=torch.int64, device=self.dist.device)
        return ops, keys

    def close(self):
        self.hs.close()


def trace_to_host(trace, stats):
    """(records sorted by ticket, keys) of a finished traced run."""
    ops, keys = trace
    n = int(stats["traced"])
    cap = ops.numel() // G.SSSPOP_DTYPE.itemsize
    if n > cap:
        raise ValueError("trace cut: %d operations, room for %d" % (n, cap))
    recs = ops.cpu().numpy().view(G.SSSPOP_DTYPE)[:n].copy()
    recs = recs[np.argsort(recs["ticket"], kind="stable")]
    return recs, keys.cpu().numpy().view(np.uint64)
