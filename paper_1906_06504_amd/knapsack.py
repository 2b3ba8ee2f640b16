"""0/1 knapsack by best-first branch and bound on the device heaps (the
application of Sec. 5.6.2): host-side preparation and the call into
heap_knapsack.  The search itself runs in the HIP library."""
from __future__ import annotations

import functools

import numpy as np
import torch

from . import gheap as G


def ratio_order(w: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Item order by value/weight descending (exact cross-multiplication),
    ties by index."""
    def cmp(i, j):
        a = int(v[i]) * int(w[j])
        b = int(v[j]) * int(w[i])
        if a != b:
            return -1 if a > b else 1
        return -1 if i < j else (1 if i > j else 0)
    return np.array(sorted(range(len(w)), key=functools.cmp_to_key(cmp)), dtype=np.int64)


class Instances:
    """Instances packed for the device (items sorted by ratio)."""

    def __init__(self, instances, device="cuda"):
        offs, ns, caps, ws, vs = [], [], [], [], []
        off = 0
        for (w, v, c) in instances:
            if len(w) > 255:
                raise ValueError("at most 255 items per instance")
            if int(np.asarray(v, dtype=np.int64).sum()) >= (1 << 18) or c >= (1 << 28):
                raise ValueError("values or capacity too large for the 35-bit bound")
            o = ratio_order(w, v)
            offs.append(off)
            ns.append(len(w))
            caps.append(c)
            ws.append(np.asarray(w, dtype=np.uint32)[o])
            vs.append(np.asarray(v, dtype=np.uint32)[o])
            off += len(w)
        self.n = len(instances)
        self.item_off = torch.from_numpy(np.array(offs, np.uint32).view(np.int32)).to(device)
        self.nitems = torch.from_numpy(np.array(ns, np.uint32).view(np.int32)).to(device)
        self.caps = torch.from_numpy(np.array(caps, np.uint64).view(np.int64)).to(device)
        cw = np.concatenate(ws) if ws else np.zeros(1, np.uint32)
        cv = np.concatenate(vs) if vs else np.zeros(1, np.uint32)
        self.w = torch.from_numpy(cw.view(np.int32)).to(device)
        self.v = torch.from_numpy(cv.view(np.int32)).to(device)


class Solver:
    """Heaps, node pools and scratch for solving a batch of instances."""

    def __init__(self, ninst: int, k: int, pool_per_inst: int = 1 << 20, device="cuda",
                 stream=None):
        self.k = k
        self.ninst = ninst
        self.pool_per_inst = pool_per_inst
        self.hs = G.HeapSet(k, [pool_per_inst] * ninst, device=device, stream=stream)
        self.snapshot = self.hs.arena.clone()
        self.pool = torch.empty(ninst * pool_per_inst, dtype=torch.int64, device=device)
        self.scratch = torch.empty(ninst * 3 * k, dtype=torch.int64, device=device)
        self.res = torch.zeros(ninst * G.KNAP_DTYPE.itemsize, dtype=torch.uint8, device=device)

    def run(self, inst: Instances, workgroups: int = 0, threads: int = 0, reset: bool = True):
        """Solve; returns the per-instance result records (numpy)."""
        if reset:
            self.hs.arena.copy_(self.snapshot)
        t = G._Tuning(workgroups, threads)
        import ctypes
        rc = self.hs.lib.heap_knapsack(self.hs.h, inst.n, inst.item_off.data_ptr(),
                                       inst.nitems.data_ptr(), inst.caps.data_ptr(),
                                       inst.w.data_ptr(), inst.v.data_ptr(), self.pool.data_ptr(),
                                       self.pool_per_inst, self.scratch.data_ptr(),
                                       self.res.data_ptr(), ctypes.byref(t))
        G._check(rc, "heap_knapsack")
        rc = self.hs.sync()
        if rc != G.GH_OK:
            raise G.GHeapError(rc, "heap_knapsack (device)")
        return self.res.cpu().numpy().view(G.KNAP_DTYPE)[: inst.n].copy()

    def close(self):
        self.hs.close()
