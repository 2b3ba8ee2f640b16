"""Shared helpers for the GPU parity tests: run an op list through the C ABI
and replay its ticket log on the oracle."""
from __future__ import annotations

import numpy as np

import oracle
from paper_1906_06504_amd import workloads as W

MAXE = np.uint64(0xFFFFFFFFFFFFFFFF)


def run_gpu(oplist, k, max_keys, workgroups=0, threads=0, heapset=None, nheaps=1):
    """Submit `oplist` on a fresh heap set (or `heapset`); returns
    (heapset, out[uint64], counts[uint32], log records).  Lists holding
    deleteMins of fewer than k entries go to the variable-count kernel."""
    import torch
    from paper_1906_06504_amd import gheap as G
    hs = heapset if heapset is not None else G.HeapSet(k, [max_keys] * nheaps)
    ops, n, keys, out, counts = G.ops_to_device(oplist)
    log = G.new_log(n)
    dels = oplist.kind == W.OP_DELETE_MIN
    var = bool(np.any(dels & (oplist.n != 0) & (oplist.n != k)))
    hs.submit(ops, n, keys, out, counts, log, workgroups=workgroups, threads=threads,
              var_delete=var)
    rc = hs.sync()
    assert rc == G.GH_OK, G.strerror(rc)
    torch.cuda.synchronize()
    return hs, G.to_host_u64(out), counts.cpu().numpy()[:n].astype(np.uint32), G.log_to_host(log, n)


def replay_and_compare(oplist, k, out_gpu, counts_gpu, log, heap=0, base_ticket=0,
                       oracle_heap=None):
    """Replay heap `heap`'s ops of `oplist` in ticket order on an oracle heap
    and compare every deleteMin output bit for bit.  Returns the oracle heap."""
    hid = oplist.heap_ids()
    sel = np.flatnonzero(hid == heap)
    tickets = log["ticket"][sel].astype(np.int64) - base_ticket
    order = sel[np.argsort(tickets, kind="stable")]
    # tickets of one heap must be exactly base, base+1, ...
    assert np.array_equal(np.sort(tickets), np.arange(sel.size)), "ticket log is not a permutation"
    oh = oracle_heap if oracle_heap is not None else oracle.OracleHeap(k)
    kinds = oplist.kind[order]
    n = oplist.n[order]
    off = oplist.off[order]
    ref_out, ref_counts = oh.replay(kinds, n, off, oplist.keys, max(oplist.out_entries, 1))
    for j, i in enumerate(order):
        if oplist.kind[i] != W.OP_DELETE_MIN:
            continue
        c = int(ref_counts[j])
        o = int(oplist.off[i])
        assert int(counts_gpu[i]) == c, "op %d: count %d != %d" % (i, counts_gpu[i], c)
        assert int(log["count"][i]) == c
        if c and not np.array_equal(out_gpu[o:o + c], ref_out[o:o + c]):
            bad = np.flatnonzero(out_gpu[o:o + c] != ref_out[o:o + c])
            raise AssertionError("op %d (ticket %d): deleteMin output differs at %d positions, first %d"
                                 % (i, log["ticket"][i], bad.size, bad[0]))
    return oh


def check_gpu_state(hs, heap, k):
    """Properties 1-3 (Sec. 3.1) on a quiescent GPU heap read back to the
    host.  Returns the live multiset (sorted)."""
    m, s, served, max_nodes, nodes, pb = hs.read_state(heap)
    live = []
    for p in range(1, m + 1):
        c = oracle.idx(p)            # node index of position p
        row = nodes[p - 1]
        assert np.all(row[:-1] <= row[1:]), "Property 2 at node %d" % c
        assert not np.any(row == MAXE), "filler inside live node %d" % c
        if c > 1:
            parent = nodes[oracle.idx(c // 2) - 1]
            assert row[0] >= parent[-1], "Property 1 at node %d" % c
        live.append(row)
    assert np.all(pb[:-1] <= pb[1:]) if pb.size > 1 else True, "Property 3 order"
    if m >= 1 and s >= 1:
        assert pb[0] >= nodes[0][-1], "Property 3 bound"
    assert s <= k - 1
    if live:
        live.append(pb)
        return np.sort(np.concatenate(live))
    return np.sort(pb)


def gpu_state_by_index(hs, heap, k):
    """GPU nodes re-indexed by tree node index (row c-1 = node c)."""
    m, s, served, max_nodes, nodes, pb = hs.read_state(heap)
    byidx = {}
    for p in range(1, m + 1):
        byidx[oracle.idx(p)] = nodes[p - 1]
    return m, s, byidx, pb


def assert_same_state(hs, heap, oh, k):
    """Heap `heap` of the GPU set equals oracle heap `oh` bit for bit: m, s,
    the partial buffer and every node (compared by tree node index)."""
    m, s, byidx, pb = gpu_state_by_index(hs, heap, k)
    assert (m, s) == (oh.m, oh.s)
    onodes, opb = oh.export()
    assert np.array_equal(pb, opb)
    for c, row in byidx.items():
        assert np.array_equal(row, onodes[c - 1]), "node %d differs" % c
