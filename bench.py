#!/usr/bin/env python3
"""Benchmark of the generalized concurrent heap on one MI355X.

Workload (one step): a single heap with node capacity k = 1024, prefilled with
2^22 uniform (u32 key, u32 id) entries as full batches (untimed, restored from
a device snapshot before every step), then a random 50/50 interleave of
inserts of U[1, 1024] fresh entries and deleteMin(1024) until 2^24 keys have
been requested, all submitted as one persistent launch with many operations in
flight.  Throughput = (keys inserted + keys returned) / device time of the
launch.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workgroups", type=int, default=0, help="operations in flight (0 = tuned default)")
    ap.add_argument("--threads", type=int, default=0, help="workgroup size (0 = tuned default)")
    ap.add_argument("--prefill", type=int, default=1 << 22)
    ap.add_argument("--requested", type=int, default=1 << 24)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain device copy of known size (for counter scaling)")
    ap.add_argument("--json-extra", action="store_true", help="print extra diagnostics")
    return ap.parse_args()


DEFAULT_SHAPE = {"workgroups": 64, "threads": 512}
TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                            "k_ops_1024_plain_heap_traffic.txt")


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; --gpus %d is not supported "
              "(run with --gpus 1)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1906_06504_amd import gheap as G
    from paper_1906_06504_amd import metrics as M
    from paper_1906_06504_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    G.load_library()
    k = 1024
    wg = args.workgroups or DEFAULT_SHAPE["workgroups"]
    th = args.threads or DEFAULT_SHAPE["threads"]

    log("generating workload: prefill %d, requested %d" % (args.prefill, args.requested))
    pre, mix, _ = W.config2(prefill=args.prefill, requested=args.requested, k=k)
    n_ins_keys = int(mix.n.sum())
    max_keys = args.prefill + n_ins_keys + k
    hs = G.HeapSet(k, [max_keys])
    stream = hs.stream

    # prefill once, keep a snapshot of the arena
    d_pre = G.ops_to_device(pre)
    hs.submit(d_pre[0], d_pre[1], d_pre[2], d_pre[3], d_pre[4], workgroups=wg, threads=th)
    rc = hs.sync()
    if rc != G.GH_OK:
        raise SystemExit("prefill failed: " + G.strerror(rc))
    snapshot = hs.arena.clone()
    torch.cuda.synchronize()
    log("prefill done: heap size %d" % hs.size())

    ops, nops, keys, out, counts = G.ops_to_device(mix)
    dlog = G.new_log(nops)

    def one_step(record):
        hs.arena.copy_(snapshot)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        hs.submit(ops, nops, keys, out, counts, dlog, workgroups=wg, threads=th)
        ev1.record(stream)
        rc = hs.sync()
        torch.cuda.synchronize()
        if rc != G.GH_OK:
            raise SystemExit("submission failed: " + G.strerror(rc))
        return ev0.elapsed_time(ev1)

    for i in range(args.warmup):
        t = one_step(False)
        log("warmup %d: %.2f ms" % (i, t))
    torch.cuda.synchronize()
    times = []
    wall0 = time.perf_counter()
    for i in range(args.steps):
        t = one_step(True)
        times.append(t)
        log("step %d: %.2f ms" % (i, t))
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0

    lg = G.log_to_host(dlog, nops)
    moved = M.keys_moved(lg)
    ms = float(np.mean(times))
    value = moved / (ms / 1e3)
    alg = int(M.algorithmic_bytes(lg, k).sum())
    achieved = alg / (ms / 1e3) / 1e9
    hz = G.clock_hz()
    lat = M.percentiles_us((lg["t_done"] - lg["t_claim"]).astype(np.int64), hz)
    t_root_sorted = np.sort(lg["t_root"].astype(np.int64))
    root_interval = float(np.median(np.diff(t_root_sorted))) * 1e6 / hz if nops > 1 else None

    result = {
        "metric": "heap keys/sec (insert+deleteMin, k=1024) vs plain; served-op p50/p99 latency",
        "value": value,
        "unit": "keys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic (SplitMix64-seeded uniform u32 keys with unique u32 ids)",
        "config": {
            "workload": "plain single heap, k=1024: prefill %d keys, then a 50/50 mix of "
                        "insert U[1,1024] and deleteMin(1024) until %d keys requested"
                        % (args.prefill, args.requested),
            "k": k, "ops": nops, "workgroups": wg, "threads": th,
            "form": "plain (one heap per launch)",
        },
        "keys_moved_per_step": moved,
        "op_latency_us": lat,
        "root_interval_us_median": root_interval,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": M.HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / M.HBM_PEAK_GBS,
            "traffic": M.stored_traffic(TRAFFIC_FILE, wg, th),
            "kernel": "gh::k_ops<1024,%d>" % th,
            "algorithmic_bytes_per_launch": alg,
        },
        "wall_s_timed_steps": wall,
    }

    if args.calib_copy:
        n = 1 << 25  # 256 MiB of int64
        a = torch.empty(n, dtype=torch.int64, device="cuda").fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("calibration copy of %d bytes done" % (n * 8))

    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        log("cpu baseline: oracle replay of the same operations on 1 core")
        oh = oracle.OracleHeap(k)
        oh.replay(pre.kind, pre.n, pre.off, pre.keys, max(pre.out_entries, 1))
        order = np.argsort(lg["ticket"], kind="stable")
        t0 = time.perf_counter()
        _, ocounts = oh.replay(mix.kind[order], mix.n[order], mix.off[order], mix.keys,
                               max(mix.out_entries, 1))
        dt = time.perf_counter() - t0
        omoved = int(mix.n.astype(np.int64).sum()) + int(ocounts.astype(np.int64).sum())
        result["cpu_baseline"] = {
            "value": omoved / dt, "unit": "keys/s", "cores": 1, "kind": "oracle",
            "sample": "the whole timed workload (%d ops, %d keys moved) replayed once in ticket "
                      "order after an untimed prefill; %.2f s" % (nops, omoved, dt),
        }
        log("cpu baseline: %.3g keys/s" % (omoved / dt))

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
