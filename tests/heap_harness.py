"""Shared helpers for the GPU parity tests: run an op list through the C ABI
and replay its ticket log on the oracle.  Op lists with 8-byte entries hold
1-D uint64 keys; those with 16-byte entries hold [n, 2] uint64 keys in the
device layout (biased key word, id word) and run on GH_I64_ID sets."""
from __future__ import annotations

import numpy as np

import oracle
from paper_1906_06504_amd import workloads as W

MAXE = np.uint64(0xFFFFFFFFFFFFFFFF)


def is_wide(a) -> bool:
    return np.asarray(a).ndim >= 2 and np.asarray(a).shape[-1] == 2


def sort_entries(a):
    """Ascending entries: integers, or [n, 2] rows ordered by word 0, then 1."""
    a = np.asarray(a, dtype=np.uint64)
    if a.ndim == 2:
        return a[np.lexsort((a[:, 1], a[:, 0]))] if a.shape[0] else a.reshape(0, 2)
    return np.sort(a)


def entries_le(a, b, wide):
    """Elementwise a <= b: integers, or [..., 2] rows ordered lexicographically."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    if wide:
        return (a[..., 0] < b[..., 0]) | ((a[..., 0] == b[..., 0]) & (a[..., 1] <= b[..., 1]))
    return a <= b


def _sorted_rows(row, wide):
    if wide:
        return bool(np.all(entries_le(row[:-1], row[1:], True)))
    return bool(np.all(row[:-1] <= row[1:]))


def _is_filler(row, wide):
    if wide:
        return np.all(row == MAXE, axis=-1)
    return row == MAXE


def run_gpu(oplist, k, max_keys, workgroups=0, threads=0, heapset=None, nheaps=1,
            bottom_up=False, shared_root=False):
    """Submit `oplist` on a fresh heap set (or `heapset`); returns
    (heapset, out, counts[uint32], log records), out as uint64 ([n, 2] for
    16-byte entries).  Lists holding deleteMins of fewer than k entries or
    inserts of more than k entries go to the general kernel."""
    import torch
    from paper_1906_06504_amd import gheap as G
    wide = is_wide(oplist.keys)
    kt = G.GH_I64_ID if wide else G.GH_U32_ID
    hs = heapset if heapset is not None else G.HeapSet(k, [max_keys] * nheaps, keytype=kt)
    ops, n, keys, out, counts = G.ops_to_device(oplist)
    log = G.new_log(n)
    dels = oplist.kind == W.OP_DELETE_MIN
    var = bool(np.any(dels & (oplist.n != 0) & (oplist.n != k)))
    multi = bool(np.any((oplist.kind == W.OP_INSERT) & (oplist.n > k)))
    hs.submit(ops, n, keys, out, counts, log, workgroups=workgroups, threads=threads,
              var_delete=var, multi_insert=multi, bottom_up=bottom_up, shared_root=shared_root)
    rc = hs.sync()
    assert rc == G.GH_OK, G.strerror(rc)
    torch.cuda.synchronize()
    return (hs, G.to_host_u64(out, hs.ewords), counts.cpu().numpy()[:n].astype(np.uint32),
            G.log_to_host(log, n))


def replay_order(oplist, log, heap=0, base_ticket=0):
    """Indices of heap `heap`'s ops in ticket order; checks that the tickets
    are exactly base, base + 1, ..."""
    hid = oplist.heap_ids()
    sel = np.flatnonzero(hid == heap)
    tickets = log["ticket"][sel].astype(np.int64) - base_ticket
    assert np.array_equal(np.sort(tickets), np.arange(sel.size)), "ticket log is not a permutation"
    return sel[np.argsort(tickets, kind="stable")]


def replay_and_compare(oplist, k, out_gpu, counts_gpu, log, heap=0, base_ticket=0,
                       oracle_heap=None):
    """Replay heap `heap`'s ops of `oplist` in ticket order on an oracle heap
    and compare every deleteMin output bit for bit.  Returns the oracle heap."""
    order = replay_order(oplist, log, heap, base_ticket)
    wide = is_wide(oplist.keys)
    oh = oracle_heap if oracle_heap is not None else oracle.OracleHeap(k, wide=wide)
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
            bad = np.flatnonzero(np.any((out_gpu[o:o + c] != ref_out[o:o + c]).reshape(c, -1), axis=1))
            raise AssertionError("op %d (ticket %d): deleteMin output differs at %d positions, first %d"
                                 % (i, log["ticket"][i], bad.size, bad[0]))
    return oh


def check_gpu_state(hs, heap, k):
    """Properties 1-3 (Sec. 3.1) on a quiescent GPU heap read back to the
    host.  Returns the live multiset (sorted)."""
    m, s, served, max_nodes, nodes, pb = hs.read_state(heap)
    wide = nodes.ndim == 3
    live = []
    for p in range(1, m + 1):
        c = oracle.idx(p)            # node index of position p
        row = nodes[p - 1]
        assert _sorted_rows(row, wide), "Property 2 at node %d" % c
        assert not np.any(_is_filler(row, wide)), "filler inside live node %d" % c
        if c > 1:
            parent = nodes[oracle.idx(c // 2) - 1]
            assert bool(entries_le(parent[-1], row[0], wide)), "Property 1 at node %d" % c
        live.append(row)
    assert _sorted_rows(pb, wide) if len(pb) > 1 else True, "Property 3 order"
    if m >= 1 and s >= 1:
        assert bool(entries_le(nodes[0][-1], pb[0], wide)), "Property 3 bound"
    assert s <= k - 1
    if live:
        live.append(pb)
        return sort_entries(np.concatenate(live))
    return sort_entries(pb)


def gpu_state_by_index(hs, heap, k):
    """GPU nodes re-indexed by tree node index (row c-1 = node c)."""
    m, s, served, max_nodes, nodes, pb = hs.read_state(heap)
    byidx = {}
    for p in range(1, m + 1):
        byidx[oracle.idx(p)] = nodes[p - 1]
    return m, s, byidx, pb


def oracle_live(oh):
    """The oracle heap's live entries, sorted."""
    onodes, opb = oh.export()
    if oh.m:
        return sort_entries(np.concatenate([onodes[oracle.idx(p) - 1] for p in range(1, oh.m + 1)]
                                           + [opb]))
    return sort_entries(opb)


def assert_same_state(hs, heap, oh, k):
    """Heap `heap` of the GPU set equals oracle heap `oh` bit for bit: m, s,
    the partial buffer and every node (compared by tree node index)."""
    m, s, byidx, pb = gpu_state_by_index(hs, heap, k)
    assert (m, s) == (oh.m, oh.s)
    onodes, opb = oh.export()
    assert np.array_equal(pb, opb)
    for c, row in byidx.items():
        assert np.array_equal(row, onodes[c - 1]), "node %d differs" % c


def flag_counts(log):
    """How many operations of a log carry each gh_logrec flag bit."""
    f = log["flags"].astype(np.uint32)
    return {b: int(np.sum((f >> b) & 1)) for b in range(8)}
