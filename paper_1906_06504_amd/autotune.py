"""Autotuner for the heap kernels: node capacity k and launch shape
(workgroup size, number of workgroups) picked by measurement.

A workload supplies `run(k, threads, workgroups) -> (milliseconds, check)`;
`check` is any value that must not depend on the shape (for the knapsack
search, the optima).  The tuner measures every candidate, refuses a winner
whose check differs from the others', and caches the choice per workload
signature in ~/.cache/gheap/autotune.json (GHEAP_TUNE_CACHE overrides).
"""
from __future__ import annotations

import json
import os
import time

from . import gheap as G

THREAD_CHOICES = (64, 128, 256, 512, 1024)


def shapes_for(k: int, threads=None):
    ts = THREAD_CHOICES if threads is None else threads
    return [t for t in ts if G.supported_shape(k, t)]


def _cache_path():
    p = os.environ.get("GHEAP_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "gheap", "autotune.json")


def load_cache():
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache):
    p = _cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        tmp = p + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, p)
    except OSError:
        pass


def tune(signature: str, run, ks, threads=None, workgroups=(0,), repeats: int = 2,
         use_cache: bool = True, log=None):
    """Measure run(k, t, wg) over the candidates; returns (best, table).
    best = {"k", "threads", "workgroups", "ms"}; table lists every candidate."""
    cache = load_cache() if use_cache else {}
    if use_cache and signature in cache:
        return cache[signature], None
    table = []
    ref_check = None
    for k in ks:
        for t in shapes_for(k, threads):
            for wg in workgroups:
                times = []
                chk = None
                for _ in range(repeats):
                    ms, chk = run(k, t, wg)
                    times.append(ms)
                ms = min(times)
                if ref_check is None:
                    ref_check = chk
                elif chk != ref_check:
                    raise RuntimeError("result changed with the launch shape: k=%d threads=%d" % (k, t))
                table.append({"k": k, "threads": t, "workgroups": wg, "ms": ms})
                if log:
                    log("tune %s: k=%d threads=%d workgroups=%d -> %.3f ms" % (signature, k, t, wg, ms))
    best = min(table, key=lambda r: r["ms"])
    if use_cache:
        cache[signature] = dict(best, when=time.time())
        save_cache(cache)
    return best, table
