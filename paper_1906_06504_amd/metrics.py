"""Measurement helpers: algorithmic bytes of a submission from its operation
log, latency percentiles, and the HBM roofline.

Algorithmic bytes are what the method has to move between HBM and the
workgroup for each operation given the path it actually took (levels and
flags come from the log), with e = 8-byte entries and node capacity k:

  insert, partial batch (n + pb <= k-1):   e*(n + pb + (n + pb)) + [root present] 2*e*k
  insert, full batch over L levels:        e*(n + pb + (n + pb - k)) + e*(2*k*L + k)
  deleteMin, no node (partial buffer):     2*e*pb
  deleteMin, one node (root only):         2*e*k
  deleteMin, refill and L merged levels:   e*k*(3 + 4*L) + 2*e*pb

(The full-batch and refill terms are the per-operation figures
e*(n + 2kD + k) and e*k*(3 + 4L) plus partial-buffer traffic.)
"""
from __future__ import annotations

import numpy as np

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published peak

FLAG_FULL = 1
FLAG_ROOT = 8
FLAG_REFILL = 16
FLAG_REJECTED = 0x40


def algorithmic_bytes(log: np.ndarray, k: int, e: int = 8) -> np.ndarray:
    """Per-operation algorithmic bytes from gh_logrec records."""
    kind = log["kind"].astype(np.int64)
    flags = log["flags"].astype(np.int64)
    levels = log["levels"].astype(np.int64)
    pb = log["pb"].astype(np.int64)
    cnt = log["count"].astype(np.int64)
    out = np.zeros(log.size, dtype=np.int64)
    ins = (kind == 0) & ((flags & FLAG_REJECTED) == 0)
    full = ins & ((flags & FLAG_FULL) != 0)
    part = ins & ~full
    n = cnt
    out[part] = e * (2 * (n[part] + pb[part])) + np.where((flags[part] & FLAG_ROOT) != 0, 2 * e * k, 0)
    out[full] = e * (n[full] + pb[full] + (n[full] + pb[full] - k)) + e * (2 * k * levels[full] + k)
    dl = kind == 1
    nonode = dl & ((flags & FLAG_ROOT) == 0)
    refill = dl & ((flags & FLAG_REFILL) != 0)
    rootonly = dl & ~nonode & ~refill
    out[nonode] = 2 * e * pb[nonode]
    out[rootonly] = 2 * e * k
    out[refill] = e * k * (3 + 4 * levels[refill]) + 2 * e * pb[refill]
    return out


def keys_moved(log: np.ndarray) -> int:
    """Keys inserted plus keys returned (rejected inserts excluded)."""
    ok = (log["flags"] & FLAG_REJECTED) == 0
    return int(log["count"][ok].astype(np.int64).sum())


def percentiles_us(ticks: np.ndarray, clock_hz: int, qs=(50, 99)) -> dict:
    if ticks.size == 0:
        return {("p%d" % q): None for q in qs}
    us = ticks.astype(np.float64) * 1e6 / clock_hz
    return {("p%d" % q): float(np.percentile(us, q)) for q in qs}


def kernel_source_hash() -> str:
    """Short hash of the HIP sources and the public header they include,
    used to tell whether stored counter readings still describe the kernel
    that is built."""
    import glob
    import hashlib
    import os
    pkg = os.path.dirname(os.path.abspath(__file__))
    files = sorted(glob.glob(os.path.join(pkg, "csrc", "*")))
    files += sorted(glob.glob(os.path.join(os.path.dirname(pkg), "include", "*.h")))
    h = hashlib.sha256()
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(path: str, workgroups: int, threads: int):
    """HBM bytes per launch recorded by a counter run (FETCH_SIZE and
    WRITE_SIZE, each scaled by a plain copy's reading), if the record matches
    the current sources and launch shape; else None."""
    import os
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if "=" in line and not line.startswith("#"):
                a, b = line.split("=", 1)
                kv[a.strip()] = b.strip()
    try:
        if kv.get("source_hash") != kernel_source_hash():
            return None
        if int(kv.get("workgroups", -1)) != workgroups or int(kv.get("threads", -1)) != threads:
            return None
        return float(kv["traffic_bytes"])
    except (KeyError, ValueError):
        return None
