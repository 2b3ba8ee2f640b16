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
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-form leg")
    ap.add_argument("--no-served", action="store_true", help="skip the served-form leg")
    ap.add_argument("--batched-heaps", type=int, default=64)
    ap.add_argument("--served-heaps", type=int, default=256)
    ap.add_argument("--served-requests", type=int, default=1 << 20)
    ap.add_argument("--served-max-log2", type=int, default=22)
    ap.add_argument("--served-slots", type=int, default=2048)
    ap.add_argument("--served-threads", type=int, default=0,
                    help="workgroup size of the served form (0 = library default)")
    ap.add_argument("--served-budget", type=int, default=1 << 20,
                    help="memory budget per heap beyond its prefill (entries)")
    ap.add_argument("--no-knapsack", action="store_true", help="skip the knapsack leg")
    ap.add_argument("--knapsack-instances", type=int, default=512)
    ap.add_argument("--no-sssp", action="store_true", help="skip the SSSP leg")
    ap.add_argument("--no-paper-table", action="store_true",
                    help="skip the insert-all-then-drain leg in the paper's key orders")
    ap.add_argument("--paper-log2n", type=int, default=26,
                    help="keys of that leg (the paper's table uses 2^29)")
    ap.add_argument("--sweep", action="store_true",
                    help="also run the parameter sweeps of the paper's experiments (node "
                         "capacity, operations in flight, partial batches); not in the default run")
    ap.add_argument("--sssp-log2v", type=int, default=20)
    ap.add_argument("--util-sweep", action="store_true",
                    help="also run the paper's initial-utilization study (heaps of 6 to 18 "
                         "levels, then ins-del pairs)")
    ap.add_argument("--util-pairs", type=int, default=1 << 15)
    ap.add_argument("--filter", action="store_true",
                    help="also time heap_filter on a 2^22-entry heap (k = 1024) at several "
                         "cut points; not in the default run")
    return ap.parse_args()


DEFAULT_SHAPE = {"workgroups": 64, "threads": 1024}
TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                            "k_ops_1024_plain_heap_traffic.txt")


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only; --gpus %d is not supported "
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
            "kernel": "gh::k_ops<1024,%d,false>" % th,
            "algorithmic_bytes_per_launch": alg,
        },
        "wall_s_timed_steps": wall,
    }

    if not args.no_batched:
        result["batched"] = run_batched(args, wg_default=wg, th=th, plain_value=value)
    if not args.no_served:
        result["served"] = run_served(args)
    if not args.no_knapsack:
        result["knapsack"] = run_knapsack(args)
    if not args.no_paper_table:
        result["paper_table"] = run_paper_table(args)
    if args.sweep:
        result["sweep"] = run_sweep(args)
    if args.util_sweep:
        result["utilization"] = run_util_sweep(args)
    if args.filter:
        result["filter"] = run_filter(args)
    sssp_graph = None
    if not args.no_sssp:
        result["sssp"], sssp_graph = run_sssp(args)

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
        order = np.argsort(lg["ticket"], kind="stable")
        times = []
        # whole-workload replays until about 10 s of timed CPU work (5 to 40)
        while len(times) < 5 or (sum(times) < 10.0 and len(times) < 40):
            oh = oracle.OracleHeap(k)
            oh.replay(pre.kind, pre.n, pre.off, pre.keys, max(pre.out_entries, 1))
            t0 = time.perf_counter()
            _, ocounts = oh.replay(mix.kind[order], mix.n[order], mix.off[order], mix.keys,
                                   max(mix.out_entries, 1))
            times.append(time.perf_counter() - t0)
        dt = float(np.median(times))
        omoved = int(mix.n.astype(np.int64).sum()) + int(ocounts.astype(np.int64).sum())
        result["cpu_baseline"] = {
            "value": omoved / dt, "unit": "keys/s", "cores": 1, "kind": "oracle",
            "sample": "the whole timed workload (%d ops, %d keys moved) replayed in ticket order "
                      "after an untimed prefill, %d times (%.1f s of timed replay); median %.2f s"
                      % (nops, omoved, len(times), sum(times), dt),
        }
        log("cpu baseline: %.3g keys/s" % (omoved / dt))
        if sssp_graph is not None:
            rowptr, col, w, src, dist = sssp_graph
            t0 = time.perf_counter()
            want = oracle.dijkstra(rowptr.size - 1, rowptr, col, w, src)
            dt = time.perf_counter() - t0
            result["sssp"]["cpu_baseline"] = {
                "value": dt * 1e3, "unit": "ms", "cores": 1, "kind": "oracle",
                "sample": "CPU Dijkstra (binary heap) on the whole graph, once",
                "distances_equal": bool(np.array_equal(dist, want)),
            }
            log("cpu baseline sssp: %.1f ms, distances equal: %s"
                % (dt * 1e3, np.array_equal(dist, want)))

    print(json.dumps(result), flush=True)


def _timed_submit(hs, d, workgroups, threads, log=None):
    import torch
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(hs.stream)
    hs.submit(d[0], d[1], d[2], d[3], d[4], log, workgroups=workgroups, threads=threads)
    ev1.record(hs.stream)
    rc = hs.sync()
    torch.cuda.synchronize()
    if rc != 0:
        raise SystemExit("submission failed: %d" % rc)
    return ev0.elapsed_time(ev1)


def run_batched(args, wg_default, th, plain_value):
    """The same total work as the plain workload (prefill 2^22, 2^24 keys
    requested, k = 1024) spread over H independent heaps: one persistent
    launch for all heaps (batched form, also replayed as a HIP graph) against
    one launch per heap (plain form)."""
    import torch
    from paper_1906_06504_amd import gheap as G
    from paper_1906_06504_amd import metrics as M
    from paper_1906_06504_amd import workloads as W
    from paper_1906_06504_amd import autotune as A
    k = 1024
    H = args.batched_heaps
    sizes = W.uneven_sizes(H, args.prefill, 6, seed=0x5EED0012)
    req_each = args.requested // H
    log("batched leg: %d heaps, prefill %d..%d (total %d), %d requested each"
        % (H, min(sizes), max(sizes), sum(sizes), req_each))
    pre, mix, pres, mixes = W.batched_mixed(H, k, sizes, req_each, seed=0x5EED0002)
    cap = max(sizes) + int(max(int(m.n.sum()) for m in mixes)) + k
    hs = G.HeapSet(k, [cap] * H, stream=torch.cuda.Stream())
    res = {}
    with torch.cuda.stream(hs.stream):
        dpre = G.ops_to_device(pre)
        _timed_submit(hs, dpre, 256, th)
        snap = hs.arena.clone()
        dmix = G.ops_to_device(mix)
        nops = dmix[1]
        dlog = G.new_log(nops)

        # launch shape by the autotuner; the results (fixed by each heap's
        # tickets) must not change with it
        def trial(kk, t, wg):
            hs.arena.copy_(snap)
            dmix[3].fill_(-1)
            torch.cuda.synchronize()
            ms = _timed_submit(hs, dmix, wg, t)
            chk = hash((dmix[3].cpu().numpy().tobytes(), dmix[4].cpu().numpy().tobytes()))
            return ms, chk
        best, table = A.tune("batched-%d-heaps" % H, trial, ks=(k,), threads=(256, 512, 1024),
                             workgroups=(H, 2 * H, 4 * H, 8 * H), repeats=2, use_cache=False,
                             log=log)
        th, wgb = best["threads"], best["workgroups"]
        times = []
        for i in range(args.warmup + args.steps):
            hs.arena.copy_(snap)
            torch.cuda.synchronize()
            t = _timed_submit(hs, dmix, wgb, th, dlog)
            if i >= args.warmup:
                times.append(t)
        lg = G.log_to_host(dlog, nops)
        moved = M.keys_moved(lg)
        ms = float(np.mean(times))
        alg = int(M.algorithmic_bytes(lg, k).sum())
        # graph replays of the same launch
        g = hs.submit_graph(dmix[0], nops, dmix[2], dmix[3], dmix[4], dlog, workgroups=wgb,
                            threads=th)
        gt = []
        for i in range(args.steps):
            hs.arena.copy_(snap)
            torch.cuda.synchronize()
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record(hs.stream)
            hs.graph_launch(g)
            ev1.record(hs.stream)
            assert hs.sync() == 0
            torch.cuda.synchronize()
            gt.append(ev0.elapsed_time(ev1))
        # plain form: every heap in its own launch, one after the other
        hs.arena.copy_(snap)
        torch.cuda.synchronize()
        plain_ms = 0.0
        plain_moved = 0
        for h in range(H):
            one = G.HeapSet(k, [cap], stream=hs.stream)
            dp = G.ops_to_device(pres[h])
            _timed_submit(one, dp, 64, th)
            dm = G.ops_to_device(mixes[h])
            l1 = G.new_log(dm[1])
            plain_ms += _timed_submit(one, dm, 64, th, l1)
            plain_moved += M.keys_moved(G.log_to_host(l1, dm[1]))
            one.close()
    value = moved / (ms / 1e3)
    res = {
        "workload": "%d heaps, k=1024, prefill sizes log-uniform over a 64x range (%d..%d, "
                    "total %d), then each a 50/50 mix of insert U[1,1024] and deleteMin(1024) "
                    "until %d keys requested" % (H, min(sizes), max(sizes), sum(sizes), req_each),
        "ops": nops, "workgroups": wgb, "threads": th, "tuning_table": table,
        "value": value, "unit": "keys/s", "ms_per_step": ms,
        "graph_ms_per_step": float(np.mean(gt)),
        "plain_one_heap_per_launch_keys_per_s": plain_moved / (plain_ms / 1e3),
        "vs_plain_per_launch": value / (plain_moved / (plain_ms / 1e3)),
        "vs_plain_single_heap_headline": value / plain_value,
        "roofline": {"bound": "hbm", "achieved": alg / (ms / 1e3) / 1e9, "peak": M.HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": alg / (ms / 1e3) / 1e9 / M.HBM_PEAK_GBS},
    }
    log("batched: %.3g keys/s (%.2f ms), plain per-heap launches %.3g keys/s"
        % (value, ms, res["plain_one_heap_per_launch_keys_per_s"]))
    hs.close()
    return res


def run_served(args):
    """Served form: H heaps (k = 256) prefilled log-uniform on
    [2^10, 2^max], a stream of requests (60% inserts of log-uniform [1, 4096]
    keys, 40% deleteMin(256), uniform heap), admitted on the device by heap
    memory.  Saturated run (all requests present at the start) gives the
    capacity; Poisson streams at 0.5x and 0.9x of it give latency."""
    import torch
    from paper_1906_06504_amd import gheap as G
    from paper_1906_06504_amd import workloads as W
    k = 256
    H = args.served_heaps
    R = args.served_requests
    log("served leg: %d heaps, %d requests" % (H, R))
    pre, reqs, sizes = W.served_stream(H, k, R, seed=0x5EED0005, rate_per_s=None,
                                       max_log2=args.served_max_log2)
    caps = W.served_capacity(sizes, extra=args.served_budget)
    hz = G.clock_hz()
    hs = G.HeapSet(k, caps, stream=torch.cuda.Stream())
    out = {"workload": "%d heaps, k=256, prefill log-uniform [2^10, 2^%d] (%d keys), %d requests: "
                       "60%% insert of log-uniform [1,4096] keys, 40%% deleteMin(256); budget per "
                       "heap prefill + %d entries" % (H, args.served_max_log2, int(sizes.sum()), R,
                                                   args.served_budget),
           "slots": args.served_slots}
    with torch.cuda.stream(hs.stream):
        dpre = G.ops_to_device(pre)
        _timed_submit(hs, dpre, 1024, 0)
        snap = hs.arena.clone()
        work = None

        def serve_once(stream_reqs):
            nonlocal work
            hs.arena.copy_(snap)
            torch.cuda.synchronize()
            r, nreq, keys, outb, recs, max_ops = G.requests_to_device(stream_reqs)
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record(hs.stream)
            work = hs.serve(r, nreq, keys, outb, recs, max_ops, work=work,
                            workgroups=args.served_slots, threads=args.served_threads)
            ev1.record(hs.stream)
            rc = hs.sync()
            torch.cuda.synchronize()
            if rc != 0:
                raise SystemExit("serving failed: %d" % rc)
            serve_once.last_out = outb
            return ev0.elapsed_time(ev1), G.recs_to_host(recs, nreq)

        def summarize(ms, recs, stream_reqs):
            adm = (recs["flags"] & G.REQ_ADMITTED) != 0
            keys = int(recs["count"][adm].astype(np.int64).sum())
            arr_ticks = stream_reqs.arrival.astype(np.float64) * hz / 1e9
            lat_us = (recs["t_done"][adm].astype(np.float64) - arr_ticks[adm]) * 1e6 / hz
            resp_us = (recs["t_resp"][adm].astype(np.float64) - arr_ticks[adm]) * 1e6 / hz
            return {"ms": ms, "keys_per_s": keys / (ms / 1e3),
                    "requests_per_s": int(adm.sum()) / (ms / 1e3),
                    "admitted": int(adm.sum()),
                    "deferred_for_memory": int(((recs["flags"] & G.REQ_DEFERRED) != 0).sum()),
                    "rejected": int(((recs["flags"] & G.REQ_REJECTED) != 0).sum()),
                    "latency_us": {"p50": float(np.percentile(lat_us, 50)),
                                   "p99": float(np.percentile(lat_us, 99))},
                    "response_latency_us": {"p50": float(np.percentile(resp_us, 50)),
                                            "p99": float(np.percentile(resp_us, 99))}}

        serve_once(reqs)  # warmup
        ms, recs = serve_once(reqs)
        sat_out = G.to_host_u64(serve_once.last_out)
        sat = summarize(ms, recs, reqs)
        out["saturated"] = sat
        log("served saturated: %.3g keys/s, %.3g req/s" % (sat["keys_per_s"], sat["requests_per_s"]))
        lam_sat = sat["requests_per_s"]
        sat_recs = recs
        import copy
        for frac in (0.5, 0.9):
            rate = frac * lam_sat
            rq = copy.copy(reqs)
            rq.arrival = W.poisson_arrivals(R, rate, seed=0x5EED0005 + int(frac * 10))
            ms, recs = serve_once(rq)
            res = summarize(ms, recs, rq)
            res["offered_requests_per_s"] = rate
            out["poisson_%.1fx" % frac] = res
            log("served at %.1fx: completion p50 %.1f us p99 %.1f us; answer p50 %.1f us p99 "
                "%.1f us" % (frac, res["latency_us"]["p50"], res["latency_us"]["p99"],
                             res["response_latency_us"]["p50"], res["response_latency_us"]["p99"]))
        # plain comparison: a sample of heaps, each heap's admitted requests
        # as its own launch (same operations, same order)
        hs.arena.copy_(snap)
        torch.cuda.synchronize()
        sample = list(range(0, H, max(1, H // 16)))
        plain_ms, plain_keys = 0.0, 0
        for h in sample:
            sel = np.flatnonzero((reqs.heap == h) & ((sat_recs["flags"] & G.REQ_ADMITTED) != 0))
            sel = sel[np.argsort(sat_recs["first_ticket"][sel], kind="stable")]
            kinds, ns, offs = [], [], []
            for i in sel:
                if reqs.kind[i] == W.OP_INSERT:
                    n = int(reqs.n[i])
                    for c in range(0, n, k):
                        kinds.append(0)
                        ns.append(min(k, n - c))
                        offs.append(int(reqs.off[i]) + c)
                else:
                    kinds.append(1)
                    ns.append(0)
                    offs.append(int(reqs.off[i]))
            if not kinds:
                continue
            ol = W.OpList(np.array(kinds, np.uint8), np.array(ns, np.uint32),
                          np.array(offs, np.uint64), reqs.keys, reqs.out_entries,
                          heap=np.full(len(kinds), h, np.uint32))
            d = G.ops_to_device(ol)
            lg = G.new_log(d[1])
            plain_ms += _timed_submit(hs, d, 64, 0, lg)
            from paper_1906_06504_amd import metrics as M
            plain_keys += M.keys_moved(G.log_to_host(lg, d[1]))
        out["plain_one_heap_per_launch_keys_per_s"] = plain_keys / (plain_ms / 1e3)
        out["vs_plain_per_launch"] = sat["keys_per_s"] / out["plain_one_heap_per_launch_keys_per_s"]
    hs.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = served_cpu_baseline(pre, reqs, sat_recs, sat_out, k, H)
    return out


def served_cpu_baseline(pre, reqs, recs, gpu_out, k, H):
    """Every heap's admitted requests of the saturated run replayed in
    ticket order on its own oracle heap (after an untimed replay of its
    prefill): one core for a sample of 16 heaps, all host cores for all
    heaps (one replay call per heap; ctypes releases the interpreter lock).
    Every deleteMin output is compared with the GPU's."""
    import concurrent.futures as cf
    import oracle
    from paper_1906_06504_amd import gheap as G
    oracle.build(force=False)
    adm = (recs["flags"] & G.REQ_ADMITTED) != 0

    def prepare(h):
        oh = oracle.OracleHeap(k)
        ps = np.flatnonzero(pre.heap == h)
        oh.replay(pre.kind[ps], pre.n[ps], pre.off[ps], pre.keys, 1)
        sel = np.flatnonzero((reqs.heap == h) & adm)
        sel = sel[np.argsort(recs["first_ticket"][sel], kind="stable")]
        dels = reqs.kind[sel] == 1
        coff = np.zeros(sel.size, np.uint64)   # compact output slots of k entries
        coff[dels] = np.arange(int(dels.sum()), dtype=np.uint64) * np.uint64(k)
        off = np.where(dels, coff, reqs.off[sel]).astype(np.uint64)
        return oh, sel, dels, off

    def replay(item):
        oh, sel, dels, off = item
        t0 = time.perf_counter()
        out, cnt = oh.replay(reqs.kind[sel], reqs.n[sel], off, reqs.keys,
                             max(1, int(dels.sum()) * k))
        dt = time.perf_counter() - t0
        moved = int(reqs.n[sel][~dels].astype(np.int64).sum()) + int(cnt.astype(np.int64).sum())
        ok = True
        for j in np.flatnonzero(dels):
            c = int(cnt[j])
            o, g = int(off[j]), int(reqs.off[sel[j]])
            if c != int(recs["count"][sel[j]]) or not np.array_equal(out[o:o + c],
                                                                       gpu_out[g:g + c]):
                ok = False
                break
        oh.close()
        return dt, moved, ok

    sample = list(range(0, H, max(1, H // 16)))
    t1, m1, ok1 = 0.0, 0, True
    for h in sample:
        dt, mv, ok = replay(prepare(h))
        t1 += dt
        m1 += mv
        ok1 = ok1 and ok
    nt = _host_threads()
    with cf.ThreadPoolExecutor(nt) as ex:
        items = list(ex.map(prepare, range(H)))
        t0 = time.perf_counter()
        rs = list(ex.map(replay, items))
        wall = time.perf_counter() - t0
    moved = sum(r[1] for r in rs)
    equal = ok1 and all(r[2] for r in rs)
    log("served cpu baseline: %.3g keys/s on 1 core (%d heaps), %.3g keys/s on %d threads "
        "(all %d heaps); outputs equal: %s" % (m1 / t1, len(sample), moved / wall, nt, H, equal))
    return {"value": moved / wall, "unit": "keys/s", "cores": nt, "kind": "oracle",
            "sample": "every heap's admitted requests of the saturated run replayed in ticket "
                      "order on %d threads (prefill replay untimed); one core: %.3g keys/s over "
                      "%d heaps" % (nt, m1 / t1, len(sample)),
            "one_core_keys_per_s": m1 / t1, "outputs_equal": bool(equal)}


def run_knapsack(args):
    """Batched form on the knapsack workload: every instance's best-first
    branch and bound on its own heap, all instances in one persistent launch
    (and replayed as a HIP graph), k and workgroup size picked by the
    autotuner; against one launch per instance (plain form)."""
    import torch
    from paper_1906_06504_amd import autotune as A
    from paper_1906_06504_amd import knapsack as KS
    from paper_1906_06504_amd import workloads as W
    N = args.knapsack_instances
    log("knapsack leg: %d instances" % N)
    inst = W.knapsack_instances(N, seed=0x5EED0004)
    dinst = KS.Instances(inst)
    pool = 1 << 20
    solvers = {}

    def run(k, t, wg):
        if k not in solvers:
            solvers[k] = KS.Solver(N, k, pool_per_inst=pool)
        s = solvers[k]
        s.hs.arena.copy_(s.snapshot)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = s.run(dinst, workgroups=wg, threads=t, reset=False)
        ms = (time.perf_counter() - t0) * 1e3
        if np.any(res["flags"] & 0x40):
            raise SystemExit("knapsack node pool overflow")
        return ms, tuple(int(b) for b in res["best"])

    best, table = A.tune("knapsack-%d-mi355x" % N, run, ks=(32, 64, 128, 256, 512, 1024),
                         threads=(64, 128, 256, 512), workgroups=(N,), repeats=2, use_cache=False,
                         log=log)
    k, t = best["k"], best["threads"]
    s = solvers[k]
    times = []
    res = None
    for _ in range(3):
        s.hs.arena.copy_(s.snapshot)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        res = s.run(dinst, workgroups=N, threads=t, reset=False)
        ev1.record()
        torch.cuda.synchronize()
        times.append(ev0.elapsed_time(ev1))
    ms = float(np.median(times))
    moved = int(res["created"].astype(np.int64).sum()) + int(res["popped"].astype(np.int64).sum())
    # plain form: each instance alone, one launch each (a sample of 64)
    sample = list(range(0, N, max(1, N // 64)))
    one = KS.Solver(1, k, pool_per_inst=pool)
    plain_ms, plain_moved = 0.0, 0
    for i in sample:
        d1 = KS.Instances([inst[i]])
        one.hs.arena.copy_(one.snapshot)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        r1 = one.run(d1, workgroups=1, threads=t, reset=False)
        ev1.record()
        torch.cuda.synchronize()
        plain_ms += ev0.elapsed_time(ev1)
        plain_moved += int(r1["created"][0]) + int(r1["popped"][0])
        if int(r1["best"][0]) != int(res["best"][i]):
            raise SystemExit("knapsack optimum differs between forms")
    one.close()
    for sv in solvers.values():
        sv.close()
    out = {
        "workload": "%d 0/1 knapsack instances, n U[40,200], w U[1,1000], v = w + U[0,100], "
                    "capacity sum(w)/2; best-first branch and bound, one heap each" % N,
        "tuned": {"k": k, "threads": t, "workgroups": N},
        "tuning_table": table,
        "ms": ms, "keys_per_s": moved / (ms / 1e3),
        "nodes_created": int(res["created"].sum()), "nodes_explored": int(res["explored"].sum()),
        "plain_one_instance_per_launch_keys_per_s": plain_moved / (plain_ms / 1e3),
        "vs_plain_per_launch": (moved / (ms / 1e3)) / (plain_moved / (plain_ms / 1e3)),
    }
    log("knapsack: k=%d threads=%d %.2f ms, %.3g keys/s (plain per launch %.3g)"
        % (k, t, ms, out["keys_per_s"], out["plain_one_instance_per_launch_keys_per_s"]))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = knapsack_cpu_baseline(inst, res["best"])
    return out


def _host_threads():
    """Worker threads for the CPU baselines: the host's cores, at most 16."""
    return max(1, min(16, os.cpu_count() or 1))


def knapsack_cpu_baseline(inst, gpu_best):
    """The oracle's dynamic program (O(n C) per instance) on one core for a
    sample of 64 instances and on all host cores for all of them (ctypes
    releases the interpreter lock during each call); the optima must equal
    the GPU's."""
    import concurrent.futures as cf
    import oracle
    oracle.build(force=False)
    sample = list(range(0, len(inst), max(1, len(inst) // 64)))
    t0 = time.perf_counter()
    for i in sample:
        w, v, c = inst[i]
        if oracle.knapsack_dp(w, v, c) != int(gpu_best[i]):
            raise SystemExit("knapsack cpu baseline: optimum differs from the GPU's")
    one = time.perf_counter() - t0
    nt = _host_threads()
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(nt) as ex:
        opt = list(ex.map(lambda x: oracle.knapsack_dp(*x), inst))
    allc = time.perf_counter() - t0
    equal = all(int(a) == int(b) for a, b in zip(opt, gpu_best))
    log("knapsack cpu baseline: DP %.1f ms per instance on 1 core; all %d instances in %.1f ms "
        "on %d threads; optima equal: %s" % (one / len(sample) * 1e3, len(inst), allc * 1e3, nt,
                                             equal))
    return {"value": allc * 1e3, "unit": "ms", "cores": nt, "kind": "oracle",
            "sample": "dynamic program for all %d instances on %d threads; one core: %.2f ms per "
                      "instance over %d instances" % (len(inst), nt, one / len(sample) * 1e3,
                                                      len(sample)),
            "one_core_ms_per_instance": one / len(sample) * 1e3,
            "optima_equal": bool(equal)}


# The paper's Table vscpu: TD-INS/TD-DEL heap, 2^29 keys inserted then all
# deleted, k = 1024, on its GPU (ms); context for the scaled run here.
PAPER_TD_MS_2E29 = {"random": 112090.0, "descending": 100163.0, "ascending": 99082.0}


def run_paper_table(args):
    """The comparison workload of the paper's Table vscpu at 2^paper_log2n
    keys: insert all keys in batches of 1024, then deleteMin(1024) until
    empty, for random, descending and ascending keys, in one launch each;
    the deleteMin outputs in ticket order must be the sorted keys."""
    import torch
    from paper_1906_06504_amd import gheap as G
    from paper_1906_06504_amd import workloads as W
    k = 1024
    N = 1 << args.paper_log2n
    out = {"workload": "insert 2^%d keys in batches of %d, then deleteMin(%d) until empty "
                       "(the paper's Table vscpu uses 2^29)" % (args.paper_log2n, k, k)}
    for order in ("random", "descending", "ascending"):
        log("paper table: %s keys, 2^%d" % (order, args.paper_log2n))
        ops = W.ordered_insert_then_drain(N, k, order, seed=0x5EED0009)
        rows = {}
        for wg in (128, 64):
            hs = G.HeapSet(k, [N + k], stream=torch.cuda.Stream())
            with torch.cuda.stream(hs.stream):
                d = G.ops_to_device(ops)
                lg = G.new_log(d[1])
                ms = _timed_submit(hs, d, wg, 0, lg)
                if wg == 128:
                    # deleteMin outputs in ticket order = all keys sorted
                    res = G.to_host_u64(d[3])
                    cnt = d[4].cpu().numpy()[:d[1]].astype(np.int64)
                    tk = G.log_to_host(lg, d[1])["ticket"]
                    dels = np.flatnonzero(ops.kind == W.OP_DELETE_MIN)
                    dels = dels[np.argsort(tk[dels], kind="stable")]
                    got = np.concatenate([res[int(ops.off[i]):int(ops.off[i]) + int(cnt[i])]
                                          for i in dels])
                    want = {"random": lambda: np.sort(ops.keys),
                            "ascending": lambda: ops.keys,
                            "descending": lambda: ops.keys[::-1]}[order]()
                    if not np.array_equal(got, want):
                        raise SystemExit("paper table: drained keys are not the sorted input")
                del d
            hs.close()
            rows["workgroups_%d" % wg] = {"ms": ms, "keys_per_s": 2 * N / (ms / 1e3)}
        best = min(r["ms"] for r in rows.values())
        rows["paper_ms_2e29_titan_x"] = PAPER_TD_MS_2E29[order]
        rows["paper_ms_scaled_to_this_n"] = PAPER_TD_MS_2E29[order] * N / (1 << 29)
        rows["speedup_vs_paper_scaled"] = rows["paper_ms_scaled_to_this_n"] / best
        out[order] = rows
        log("paper table %s: %.1f ms (paper, scaled: %.1f ms)"
            % (order, best, rows["paper_ms_scaled_to_this_n"]))
    return out


def run_filter(args):
    """heap_filter (the garbage collection of branch and bound) on a heap of
    2^22 entries, k = 1024, built from a sorted array and then shuffled by a
    concurrent mix of 2^20 requested keys; cut at the 10th, 50th and 90th
    percentile of its entries.  Each cut starts from the same state (an
    arena snapshot) and is timed with HIP events on the heap's stream."""
    import torch
    from paper_1906_06504_amd import gheap as G
    from paper_1906_06504_amd import workloads as W
    k, n = 1024, 1 << 22
    keys = np.sort(W.prefill_ops(n, k, 0x5EED0002).keys)
    hs = G.HeapSet(k, [n + (1 << 20)], stream=torch.cuda.Stream())
    with torch.cuda.stream(hs.stream):
        hs.build(0, G.to_device_u64(keys))
        mix = W.mixed_ops(1 << 20, k, seed=77, first_id=n)
        d = G.ops_to_device(mix)
        hs.submit(*d[:5], workgroups=64)
    if hs.sync() != 0:
        raise SystemExit("filter leg: setup failed")
    torch.cuda.synchronize()
    m, s, _, _, nodes, pb = hs.read_state(0)
    live = np.sort(np.concatenate([nodes[:m].reshape(-1), pb]))
    snap = hs.arena.clone()
    out = {"workload": "filter of a %d-entry heap, k = %d" % (live.size, k)}
    work = None
    for q in (0.1, 0.5, 0.9):
        bound = int(live[int(q * (live.size - 1))])
        times = []
        for rep in range(4):
            hs.arena.copy_(snap)
            torch.cuda.synchronize()
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record(hs.stream)
            kept, work = hs.filter(0, bound, work)
            ev1.record(hs.stream)
            if hs.sync() != 0:
                raise SystemExit("filter leg: filter failed")
            torch.cuda.synchronize()
            times.append(ev0.elapsed_time(ev1))
            if int(kept.item()) != int(np.sum(live < np.uint64(bound))):
                raise SystemExit("filter leg: wrong number kept")
        ms = float(np.median(times[1:]))
        out["q%02d" % int(q * 100)] = {"kept": int(kept.item()), "ms": ms,
                                       "entries_per_s": live.size / (ms / 1e3)}
        log("filter at the %d%% point: kept %d of %d in %.3f ms"
            % (int(q * 100), int(kept.item()), live.size, ms))
    hs.close()
    return out


def run_util_sweep(args):
    """The paper's initial-utilization study (Sec. 5, heap utilization):
    the heap starts with 2^L full nodes (L = 6 .. 18 levels, 64K to 256M
    entries at k = 1024), then 128 workgroups run ins-del pairs (insert 1024
    random entries, deleteMin 1024), so the heap keeps its size.  The paper
    runs 2^18 pairs; here 2^15 (--util-pairs) and the time per pair is
    reported.  The initial heap is a bulk build of a sorted array (a sorted
    array is a generalized heap, Sec. 3.1), generated and sorted on the
    device from a seeded generator; keys are 31 bits so that signed and
    unsigned order agree."""
    import torch
    from paper_1906_06504_amd import gheap as G
    from paper_1906_06504_amd import workloads as W
    k, wg, pairs = 1024, 128, args.util_pairs
    rng = np.random.default_rng(0x5EED000C)
    out = {"workload": "initial heap of 2^L nodes (k = 1024), then %d ins-del pairs on %d "
                       "workgroups" % (pairs, wg), "rows": []}
    for L in (6, 8, 10, 12, 14, 16, 18):
        n0 = k << L
        ins_keys = ((rng.integers(0, 1 << 31, pairs * k, dtype=np.uint64) << np.uint64(32))
                    | np.arange(n0, n0 + pairs * k, dtype=np.uint64))
        ops = W.build_oplist([W.OP_INSERT, W.OP_DELETE_MIN] * pairs, [k, 0] * pairs,
                             lambda c: ins_keys[:c], k)
        hs = G.HeapSet(k, [n0 + 4 * wg * k], stream=torch.cuda.Stream())
        with torch.cuda.stream(hs.stream):
            gen = torch.Generator(device="cuda")
            gen.manual_seed(0x5EED000D + L)
            ent = torch.randint(0, 1 << 31, (n0,), generator=gen, device="cuda",
                                dtype=torch.int64)
            ent = torch.sort((ent << 32) | torch.arange(n0, device="cuda",
                                                        dtype=torch.int64)).values
            hs.build(0, ent)
            d = G.ops_to_device(ops)
        if hs.sync() != 0:
            raise SystemExit("utilization sweep: build failed")
        del ent
        with torch.cuda.stream(hs.stream):
            ms = _timed_submit(hs, d, wg, 0)
        size = hs.size(0)
        hs.close()
        del d, hs
        torch.cuda.empty_cache()
        if size != n0:
            raise SystemExit("utilization sweep: heap size %d after the pairs, expected %d"
                             % (size, n0))
        out["rows"].append({"levels": L, "initial_keys": n0, "ms": ms,
                            "us_per_pair": ms * 1e3 / pairs})
        log("utilization sweep: %d levels (%d keys): %.1f ms, %.2f us per pair"
            % (L, n0, ms, ms * 1e3 / pairs))
    return out


def run_sweep(args):
    """The shapes of the paper's parameter studies on this GPU, on the
    insert-all-then-drain workload with random keys (2^24 keys): node
    capacity k (default workgroup size for each k, 64 operations in flight),
    the number of operations in flight at k = 1024, and full against partial
    insert batches (batches of k, or sizes uniform on [1, k])."""
    import torch
    from paper_1906_06504_amd import gheap as G
    from paper_1906_06504_amd import workloads as W
    N = 1 << 24

    def timed(ops, k, wg, th):
        hs = G.HeapSet(k, [N + k], stream=torch.cuda.Stream())
        with torch.cuda.stream(hs.stream):
            d = G.ops_to_device(ops)
            ms = _timed_submit(hs, d, wg, th)
            del d
        hs.close()
        return ms

    out = {"workload": "insert 2^24 random keys, then deleteMin(k) until empty"}
    rows = []
    for k in (64, 128, 256, 512, 1024):
        ops = W.ordered_insert_then_drain(N, k, "random", seed=0x5EED000A)
        ms = timed(ops, k, 64, 0)
        rows.append({"k": k, "workgroups": 64, "ms": ms, "keys_per_s": 2 * N / (ms / 1e3)})
        log("sweep k=%d: %.1f ms" % (k, ms))
    out["node_capacity"] = rows
    rows = []
    ops = W.ordered_insert_then_drain(N, 1024, "random", seed=0x5EED000A)
    for wg in (1, 4, 16, 32, 64, 128, 256):
        ms = timed(ops, 1024, wg, 512)
        rows.append({"k": 1024, "workgroups": wg, "ms": ms, "keys_per_s": 2 * N / (ms / 1e3)})
        log("sweep workgroups=%d: %.1f ms" % (wg, ms))
    out["operations_in_flight"] = rows
    # partial batches: the same keys inserted in batches of uniform size
    st = W.Stream(0x5EED000B)
    sizes, acc = [], 0
    while acc < N:
        b = int(min(st.uniform_int(1, 1024, 1)[0], N - acc))
        sizes.append(b)
        acc += b
    n_del = N // 1024 + 1
    kinds = [W.OP_INSERT] * len(sizes) + [W.OP_DELETE_MIN] * n_del
    part = W.build_oplist(kinds, sizes + [0] * n_del, W._keys_with_ids(W.Stream(0x5EED000A), 0),
                          1024)
    ms_full = out["operations_in_flight"][4]["ms"]
    ms_part = timed(part, 1024, 64, 512)
    out["partial_batches"] = {"full_batches_ms": ms_full, "uniform_1_to_k_batches_ms": ms_part,
                              "insert_ops_full": N // 1024, "insert_ops_partial": len(sizes)}
    log("sweep partial batches: %.1f ms vs full %.1f ms" % (ms_part, ms_full))
    return out


def run_sssp(args):
    """SSSP on one shared heap (lazy Dijkstra, many workgroups popping k = 512
    entries at a time): run time, edges per second, and the split of device
    time between heap operations and edge relaxation."""
    import torch
    from paper_1906_06504_amd import gheap as GH
    from paper_1906_06504_amd import sssp as SP
    from paper_1906_06504_amd import workloads as W
    V = 1 << args.sssp_log2v
    log("sssp leg: generating graph with %d vertices" % V)
    rowptr, col, w, src, k = W.config3(V)
    g = SP.Graph(rowptr, col, w)
    table = []
    best = None
    dist = None
    for t in (256, 512, 1024):
        for wg in (8, 16, 32, 64, 128, 256):
            sol = SP.Solver(g, k, workgroups=wg, threads=t, stream=torch.cuda.Stream())
            sol.run(src)   # warm
            times, stats = [], None
            for _ in range(3):
                ev0 = torch.cuda.Event(enable_timing=True)
                ev1 = torch.cuda.Event(enable_timing=True)
                ev0.record(sol.hs.stream)
                sol.launch(src)
                ev1.record(sol.hs.stream)
                rc = sol.hs.sync()
                if rc != 0:
                    raise SystemExit("sssp failed: %d" % rc)
                torch.cuda.synchronize()
                times.append(ev0.elapsed_time(ev1))
            d = sol.dist.cpu().numpy().view(np.uint32)[:V].copy()
            stats = sol.stats.cpu().numpy().view(GH.SSSP_DTYPE)[0]
            if dist is None:
                dist = d
            elif not np.array_equal(d, dist):
                raise SystemExit("sssp distances differ between launch shapes")
            ms = float(np.median(times))
            row = {"threads": t, "workgroups": wg, "ms": ms}
            table.append(row)
            log("sssp threads=%d workgroups=%d: %.2f ms" % (t, wg, ms))
            if best is None or ms < best[0]["ms"]:
                best = (row, stats)
            sol.close()
    row, st = best
    ht, rt = int(st["heap_ticks"]), int(st["relax_ticks"])
    moved = int(st["pushed"]) + 1 + int(st["popped"])
    reached = int(np.sum(dist != 0xFFFFFFFF))
    out = {
        "workload": "SSSP from vertex 0, V=2^%d, out-degree Poisson(8), w U[1,1000], E=%d, k=%d; "
                    "lazy deletion on one shared heap" % (args.sssp_log2v, g.E, k),
        "best": row, "table": table,
        "ms": row["ms"],
        "edges_per_s": g.E / (row["ms"] / 1e3),
        "heap_keys_per_s": moved / (row["ms"] / 1e3),
        "heap_time_share": ht / max(1, ht + rt),
        "popped": int(st["popped"]), "stale": int(st["stale"]), "pushed": int(st["pushed"]),
        "reexpanded": int(st["popped"]) - int(st["stale"]) - reached,
        "heap_ops": int(st["heap_ops"]), "reached": reached,
    }
    log("sssp: %.2f ms, %.3g edges/s, heap share %.2f" % (row["ms"], out["edges_per_s"],
                                                         out["heap_time_share"]))
    return out, (rowptr, col, w, src, dist)


if __name__ == "__main__":
    main()
