"""0/1 knapsack by best-first branch and bound on the device heaps (the
application of Sec. 5.7.2): host-side preparation and the call into
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


# Largest value sum an instance may have, by key type: the 8-byte entry packs
# a 35-bit bound, the 16-byte one is limited by the node pool's 28-bit fields.
VALUE_SUM_LIMIT = {G.GH_U32_ID: 1 << 18, G.GH_I64_ID: 1 << 28}


class Instances:
    """Instances packed for the device (items sorted by ratio).  With
    check=True instances beyond the library's limits raise here; otherwise
    they reach the device, which refuses them (result flag bit 5)."""

    def __init__(self, instances, device="cuda", keytype: int = G.GH_I64_ID, check: bool = True):
        offs, ns, caps, ws, vs = [], [], [], [], []
        off = 0
        for (w, v, c) in instances:
            if check and len(w) > 255:
                raise ValueError("at most 255 items per instance")
            if check and (int(np.asarray(v, dtype=np.int64).sum()) >= VALUE_SUM_LIMIT[keytype]
                          or c >= (1 << 28)):
                raise ValueError("values or capacity too large for the entry's bound")
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
                 stream=None, keytype: int = G.GH_I64_ID):
        self.k = k
        self.ninst = ninst
        self.pool_per_inst = pool_per_inst
        self.hs = G.HeapSet(k, [pool_per_inst] * ninst, device=device, stream=stream,
                            keytype=keytype)
        self.snapshot = self.hs.arena.clone()
        self.pool = torch.empty(ninst * pool_per_inst, dtype=torch.int64, device=device)
        self.scratch = torch.empty(ninst * 3 * k * self.hs.ewords, dtype=torch.int64,
                                   device=device)
        self.res = torch.zeros(ninst * G.KNAP_DTYPE.itemsize, dtype=torch.uint8, device=device)

    def launch(self, inst: Instances, workgroups: int = 0, threads: int = 0, reset: bool = True,
               gc_min: int = 0):
        """Queue the solve on the set's stream (no wait).  gc_min > 0 turns
        on garbage collection of heaps holding at least gc_min entries."""
        import ctypes
        if reset:
            self.hs.arena.copy_(self.snapshot)
        t = G._Tuning(workgroups, threads)
        rc = self.hs.lib.heap_knapsack(self.hs.h, inst.n, inst.item_off.data_ptr(),
                                       inst.nitems.data_ptr(), inst.caps.data_ptr(),
                                       inst.w.data_ptr(), inst.v.data_ptr(), self.pool.data_ptr(),
                                       self.pool_per_inst, self.scratch.data_ptr(),
                                       self.res.data_ptr(), int(gc_min), ctypes.byref(t))
        G._check(rc, "heap_knapsack")

    def results(self, n: int):
        return self.res.cpu().numpy().view(G.KNAP_DTYPE)[:n].copy()

    def run(self, inst: Instances, workgroups: int = 0, threads: int = 0, reset: bool = True,
            gc_min: int = 0, allow_device_error: bool = False):
        """Solve; returns the per-instance result records (numpy)."""
        self.launch(inst, workgroups, threads, reset, gc_min)
        rc = self.hs.sync()
        if rc != G.GH_OK and not allow_device_error:
            raise G.GHeapError(rc, "heap_knapsack (device)")
        return self.results(inst.n)

    def close(self):
        self.hs.close()
